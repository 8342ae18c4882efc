// Nested-dissection ordering and multifrontal LU (no pivoting) of the
// mean-parameter preconditioner, producing the inverted-block data of the
// level-scheduled triangular solves.  See ndfact.h for the data layout.
#include "ndfact.h"

#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

namespace lrc {
namespace {

using clk = std::chrono::steady_clock;
static double secs(clk::time_point a) {
  return std::chrono::duration<double>(clk::now() - a).count();
}

// ------------------------------------------------------------------ graph of P + P^T
struct Graph {
  int64_t n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  int deg(int v) const { return int(xadj[v + 1] - xadj[v]); }
};

static Graph symmetric_graph(const CsrHost& P) {
  const int64_t n = P.n;
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
      int64_t j = P.col[e];
      if (j == i) continue;
      cnt[i + 1]++;
      cnt[j + 1]++;
    }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> tmp(cnt[n]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
      int64_t j = P.col[e];
      if (j == i) continue;
      tmp[fill[i]++] = int32_t(j);
      tmp[fill[j]++] = int32_t(i);
    }
  Graph g;
  g.n = n;
  g.xadj.assign(n + 1, 0);
  g.adj.reserve(tmp.size());
  for (int64_t i = 0; i < n; ++i) {
    auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
    std::sort(b, e);
    auto u = std::unique(b, e);
    g.adj.insert(g.adj.end(), b, u);
    g.xadj[i + 1] = int64_t(g.adj.size());
  }
  return g;
}

// ------------------------------------------------------------------ nested dissection
struct NDBuilder {
  const Graph& g;
  int leaf;
  std::vector<int32_t> part;     // subset id of each vertex
  std::vector<int32_t> level;    // BFS level scratch
  int next_part = 1;
  std::vector<int32_t> order;    // new -> old, filled in post-order
  std::vector<int32_t> j0, ns, parent;

  NDBuilder(const Graph& g_, int leaf_) : g(g_), leaf(leaf_) {
    part.assign(g.n, 0);
    level.assign(g.n, -1);
  }

  int new_node(const std::vector<int32_t>& verts, const std::vector<int>& children) {
    int id = int(j0.size());
    j0.push_back(int32_t(order.size()));
    ns.push_back(int32_t(verts.size()));
    parent.push_back(-1);
    for (int c : children) parent[c] = id;
    order.insert(order.end(), verts.begin(), verts.end());
    return id;
  }

  // BFS restricted to vertices with part == pid; fills level[], returns the
  // level lists (vertices in BFS order) and their count.
  void bfs(int32_t root, int32_t pid, std::vector<int32_t>& q, std::vector<int32_t>& lstart) {
    q.clear();
    lstart.clear();
    q.push_back(root);
    level[root] = 0;
    lstart.push_back(0);
    size_t head = 0;
    int cur = 0;
    while (head < q.size()) {
      int32_t v = q[head++];
      if (level[v] != cur) {
        cur = level[v];
        lstart.push_back(int32_t(head - 1));
      }
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
        int32_t u = g.adj[e];
        if (part[u] == pid && level[u] < 0) {
          level[u] = level[v] + 1;
          q.push_back(u);
        }
      }
    }
    lstart.push_back(int32_t(q.size()));
  }

  void clear_levels(const std::vector<int32_t>& q) {
    for (int32_t v : q) level[v] = -1;
  }

  // Recursively dissect `verts` (all tagged with a fresh part id by the
  // caller); returns the tree roots created for them.
  std::vector<int> rec(std::vector<int32_t> verts, int32_t pid) {
    std::vector<int> roots;
    if (verts.empty()) return roots;
    // connected components
    std::vector<int32_t> q, ls;
    std::vector<std::vector<int32_t>> comps;
    for (int32_t v : verts) {
      if (level[v] >= 0) continue;
      bfs(v, pid, q, ls);
      comps.push_back(q);
    }
    for (auto& c : comps) clear_levels(c);
    for (auto& comp : comps) {
      if (int(comp.size()) <= leaf) {
        roots.push_back(new_node(comp, {}));
        continue;
      }
      // pseudo-peripheral start vertex
      int32_t start = comp[0];
      for (int32_t v : comp)
        if (g.deg(v) < g.deg(start)) start = v;
      int ecc = -1;
      for (int it = 0; it < 5; ++it) {
        bfs(start, pid, q, ls);
        int e = int(ls.size()) - 2;
        int32_t cand = q[ls[e]];
        for (int32_t k = ls[e]; k < ls[e + 1]; ++k)
          if (g.deg(q[k]) < g.deg(cand)) cand = q[k];
        clear_levels(q);
        if (e <= ecc) break;
        ecc = e;
        start = cand;
      }
      bfs(start, pid, q, ls);
      const int E = int(ls.size()) - 2;   // max level
      if (E < 2) {                         // (near) clique: keep dense
        clear_levels(q);
        roots.push_back(new_node(comp, {}));
        continue;
      }
      // level L with |levels < L| closest to half
      int L = 1;
      int64_t best = INT64_MAX;
      const int64_t half = int64_t(comp.size()) / 2;
      for (int l = 1; l < E; ++l) {
        int64_t below = ls[l];
        int64_t d = std::llabs(below - half);
        if (d < best) { best = d; L = l; }
      }
      std::vector<int32_t> A, B, S;
      for (size_t k = 0; k < q.size(); ++k) {
        int32_t v = q[k];
        int lv = level[v];
        if (lv < L) A.push_back(v);
        else if (lv > L) B.push_back(v);
        else {
          bool touches_next = false;
          for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            int32_t u = g.adj[e];
            if (part[u] == pid && level[u] == L + 1) { touches_next = true; break; }
          }
          (touches_next ? S : A).push_back(v);
        }
      }
      clear_levels(q);
      int32_t pa = next_part++, pb = next_part++;
      for (int32_t v : A) part[v] = pa;
      for (int32_t v : B) part[v] = pb;
      for (int32_t v : S) part[v] = -1;
      std::vector<int> ch = rec(std::move(A), pa);
      std::vector<int> chb = rec(std::move(B), pb);
      ch.insert(ch.end(), chb.begin(), chb.end());
      roots.push_back(new_node(S, ch));
    }
    return roots;
  }
};

// ------------------------------------------------------------------ dense helpers
// C[r][c] -= sum_p A[r][p] * B[p][c] for a row-major block; lda/ldb/ldc strides.
static void gemm_sub(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double* C, int64_t ldc, bool par) {
  if (M == 0 || N == 0 || K == 0) return;
#pragma omp parallel for schedule(static) if (par && M * N * K > (1 << 18))
  for (int64_t r = 0; r < M; ++r) {
    double* __restrict c = C + r * ldc;
    const double* __restrict a = A + r * lda;
    for (int64_t p = 0; p < K; ++p) {
      const double ap = a[p];
      if (ap == 0.0) continue;
      const double* __restrict b = B + p * ldb;
      for (int64_t j = 0; j < N; ++j) c[j] -= ap * b[j];
    }
  }
}

// In-place partial LU (no pivoting) of the first k pivots of the f x f
// row-major matrix F.  Returns the index of a bad pivot or -1.
static int64_t partial_lu(double* F, int64_t f, int64_t k, double tiny, bool par) {
  const int64_t NB = 48;
  for (int64_t kb = 0; kb < k; kb += NB) {
    const int64_t ke = std::min(k, kb + NB);
    // panel: columns [kb, ke), all rows >= kb
    for (int64_t p = kb; p < ke; ++p) {
      const double piv = F[p * f + p];
      if (!(std::fabs(piv) > tiny)) return p;
      const double inv = 1.0 / piv;
      for (int64_t r = p + 1; r < f; ++r) {
        double* row = F + r * f;
        const double l = row[p] * inv;
        row[p] = l;
        if (l == 0.0) continue;
        const double* prow = F + p * f;
        for (int64_t c = p + 1; c < ke; ++c) row[c] -= l * prow[c];
      }
    }
    if (ke >= f) continue;
    // U12 rows [kb, ke), cols [ke, f): forward substitution with the unit panel
    for (int64_t p = kb; p < ke; ++p)
      for (int64_t r = p + 1; r < ke; ++r) {
        const double l = F[r * f + p];
        if (l == 0.0) continue;
        double* row = F + r * f;
        const double* prow = F + p * f;
        for (int64_t c = ke; c < f; ++c) row[c] -= l * prow[c];
      }
    // trailing update
    gemm_sub(f - ke, f - ke, ke - kb, F + ke * f + kb, f, F + kb * f + ke, f, F + ke * f + ke, f,
             par);
  }
  return -1;
}

}  // namespace

bool nd_order(const CsrHost& P, int leaf_size, std::vector<int32_t>* perm,
              std::vector<int32_t>* j0, std::vector<int32_t>* ns,
              std::vector<int32_t>* parent, std::string* err) {
  if (P.n <= 0 || int64_t(P.rowptr.size()) != P.n + 1) {
    if (err) *err = "nd_order: bad CSR";
    return false;
  }
  Graph g = symmetric_graph(P);
  NDBuilder b(g, std::max(1, leaf_size));
  std::vector<int32_t> all(P.n);
  std::iota(all.begin(), all.end(), 0);
  int32_t pid = b.next_part++;
  for (auto v : all) b.part[v] = pid;
  b.rec(std::move(all), pid);
  if (int64_t(b.order.size()) != P.n) {
    if (err) *err = "nd_order: ordering lost vertices";
    return false;
  }
  *perm = std::move(b.order);
  *j0 = std::move(b.j0);
  *ns = std::move(b.ns);
  *parent = std::move(b.parent);
  return true;
}

int nd_factor(const CsrHost& P, int leaf_size, int nthreads, SupernodalFactor* out,
              std::string* err) {
  auto t0 = clk::now();
  SupernodalFactor& F = *out;
  F = SupernodalFactor();
  const int64_t n = P.n;
  if (n <= 0 || n > INT32_MAX) { *err = "nd_factor: bad size"; return -1; }
  if (nthreads > 0) omp_set_num_threads(nthreads);
  if (!nd_order(P, leaf_size, &F.perm, &F.j0, &F.ns, &F.parent, err)) return -1;
  F.n = n;
  F.nsn = int(F.j0.size());
  const int S = F.nsn;
  F.iperm.assign(n, 0);
  for (int64_t j = 0; j < n; ++j) F.iperm[F.perm[j]] = int32_t(j);

  // tree levels
  std::vector<std::vector<int>> children(S);
  for (int s = 0; s < S; ++s)
    if (F.parent[s] >= 0) children[F.parent[s]].push_back(s);
  F.height.assign(S, 0);
  for (int s = 0; s < S; ++s)            // ids are post-ordered: children first
    for (int c : children[s]) F.height[s] = std::max(F.height[s], F.height[c] + 1);
  F.depth.assign(S, 0);
  for (int s = S - 1; s >= 0; --s)
    if (F.parent[s] >= 0) F.depth[s] = F.depth[F.parent[s]] + 1;
  F.nlev_fwd = 1 + *std::max_element(F.height.begin(), F.height.end());
  F.nlev_bwd = 1 + *std::max_element(F.depth.begin(), F.depth.end());

  // symbolic: boundary sets
  Graph g = symmetric_graph(P);
  std::vector<std::vector<int32_t>> bnd(S);
  {
    std::vector<int32_t> marker(n, -1);
    for (int s = 0; s < S; ++s) {
      const int32_t a = F.j0[s], e = F.j0[s] + F.ns[s];
      auto& B = bnd[s];
      for (int32_t j = a; j < e; ++j) {
        int32_t v = F.perm[j];
        for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
          int32_t u = F.iperm[g.adj[k]];
          if (u >= e && marker[u] != s) { marker[u] = s; B.push_back(u); }
        }
      }
      for (int c : children[s])
        for (int32_t u : bnd[c])
          if (u >= e && marker[u] != s) { marker[u] = s; B.push_back(u); }
      std::sort(B.begin(), B.end());
    }
  }
  F.nb.assign(S, 0);
  F.bnd_off.assign(S + 1, 0);
  for (int s = 0; s < S; ++s) {
    F.nb[s] = int32_t(bnd[s].size());
    F.bnd_off[s + 1] = F.bnd_off[s] + F.nb[s];
  }
  F.bnd.reserve(F.bnd_off[S]);
  for (int s = 0; s < S; ++s) F.bnd.insert(F.bnd.end(), bnd[s].begin(), bnd[s].end());

  F.fw_off.assign(S + 1, 0);
  F.front_off.assign(S + 1, 0);
  F.cb_off.assign(S + 1, 0);
  for (int s = 0; s < S; ++s) {
    int64_t f = int64_t(F.ns[s]) + F.nb[s];
    F.fw_off[s + 1] = F.fw_off[s] + f * F.ns[s];
    F.front_off[s + 1] = F.front_off[s] + f;
    F.cb_off[s + 1] = F.cb_off[s] + F.nb[s];
    F.max_front = std::max(F.max_front, f);
    F.factor_flops += 2.0 / 3.0 * double(F.ns[s]) * F.ns[s] * F.ns[s] +
                      2.0 * double(F.ns[s]) * F.ns[s] * F.nb[s] +
                      2.0 * double(F.nb[s]) * F.nb[s] * F.ns[s];
  }
  F.bw_off = F.fw_off;   // same sizes: f * ns
  F.fw.assign(F.fw_off[S], 0.0);
  F.bw.assign(F.bw_off[S], 0.0);
  F.dense_entries = 2.0 * double(F.fw_off[S]);
  F.seconds_order = secs(t0);

  // transpose of P for column access
  auto t1 = clk::now();
  std::vector<int64_t> tptr(n + 1, 0);
  for (int64_t e = 0; e < P.rowptr[n]; ++e) tptr[P.col[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  std::vector<int32_t> trow(P.rowptr[n]);
  std::vector<double> tval(P.rowptr[n]);
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
        int64_t c = P.col[e];
        trow[fill[c]] = int32_t(i);
        tval[fill[c]++] = P.val[e];
      }
  }
  double pmax = 0.0;
  for (double v : P.val) {
    if (!std::isfinite(v)) { *err = "nd_factor: non-finite entry in P"; return -1; }
    pmax = std::max(pmax, std::fabs(v));
  }
  const double tiny = 1e-14 * std::max(pmax, 1e-300);

  // numeric multifrontal LU, level by level (children before parents)
  std::vector<std::vector<double>> cb(S);
  std::vector<std::vector<int>> by_height(F.nlev_fwd);
  for (int s = 0; s < S; ++s) by_height[F.height[s]].push_back(s);
  const int nthr = std::max(1, omp_get_max_threads());
  std::vector<std::vector<int32_t>> posmap(nthr, std::vector<int32_t>());
  int bad = -1;
  std::string bad_msg;

  auto factor_one = [&](int s, bool par) -> int {
    int tid = par ? 0 : omp_get_thread_num();
    auto& pos = posmap[tid];
    if (pos.empty()) pos.assign(n, -1);
    const int64_t nsv = F.ns[s], nbv = F.nb[s], f = nsv + nbv;
    const int32_t a = F.j0[s], e = a + int32_t(nsv);
    const int32_t* B = F.bnd.data() + F.bnd_off[s];
    for (int64_t p = 0; p < nsv; ++p) pos[a + p] = int32_t(p);
    for (int64_t p = 0; p < nbv; ++p) pos[B[p]] = int32_t(nsv + p);
    std::vector<double> Fm(size_t(f * f), 0.0);
    // original entries with min(row, col) in own(s)
    for (int32_t j = a; j < e; ++j) {
      const int32_t old = F.perm[j];
      const int64_t r = pos[j];
      for (int64_t k = P.rowptr[old]; k < P.rowptr[old + 1]; ++k) {
        int32_t c = F.iperm[P.col[k]];
        if (c >= a) Fm[r * f + pos[c]] += P.val[k];
      }
      for (int64_t k = tptr[old]; k < tptr[old + 1]; ++k) {
        int32_t rr = F.iperm[trow[k]];
        if (rr >= e) Fm[int64_t(pos[rr]) * f + pos[j]] += tval[k];
      }
    }
    // extend-add of the children's update matrices
    for (int c : children[s]) {
      const int64_t nc = F.nb[c];
      const int32_t* Bc = F.bnd.data() + F.bnd_off[c];
      const double* U = cb[c].data();
      for (int64_t x = 0; x < nc; ++x) {
        double* row = Fm.data() + int64_t(pos[Bc[x]]) * f;
        for (int64_t y = 0; y < nc; ++y) row[pos[Bc[y]]] += U[x * nc + y];
      }
      std::vector<double>().swap(cb[c]);
    }
    for (int64_t p = 0; p < nsv; ++p) pos[a + p] = -1;
    for (int64_t p = 0; p < nbv; ++p) pos[B[p]] = -1;
    int64_t badp = partial_lu(Fm.data(), f, nsv, tiny, par);
    if (badp >= 0) return int(a + badp);
    // update matrix for the parent
    cb[s].resize(size_t(nbv * nbv));
    for (int64_t x = 0; x < nbv; ++x)
      std::memcpy(cb[s].data() + x * nbv, Fm.data() + (nsv + x) * f + nsv, sizeof(double) * nbv);
    // inverses of the diagonal blocks
    std::vector<double> Li(size_t(nsv * nsv), 0.0), Ui(size_t(nsv * nsv), 0.0);
    for (int64_t i = 0; i < nsv; ++i) {              // Linv row i = e_i - sum_p L[i][p] Linv row p
      double* ri = Li.data() + i * nsv;
      ri[i] = 1.0;
      for (int64_t p = 0; p < i; ++p) {
        const double l = Fm[i * f + p];
        if (l == 0.0) continue;
        const double* rp = Li.data() + p * nsv;
        for (int64_t j = 0; j <= p; ++j) ri[j] -= l * rp[j];
      }
    }
    for (int64_t i = nsv - 1; i >= 0; --i) {         // Uinv row i
      double* ri = Ui.data() + i * nsv;
      const double dinv = 1.0 / Fm[i * f + i];
      ri[i] = 1.0;
      for (int64_t p = i + 1; p < nsv; ++p) {
        const double u = Fm[i * f + p];
        if (u == 0.0) continue;
        const double* rp = Ui.data() + p * nsv;
        for (int64_t j = p; j < nsv; ++j) ri[j] -= u * rp[j];
      }
      for (int64_t j = i; j < nsv; ++j) ri[j] *= dinv;
    }
    // Fw (column-major, f x ns): [Linv ; -L21 Linv]
    double* fw = F.fw.data() + F.fw_off[s];
    for (int64_t i = 0; i < nsv; ++i)
      for (int64_t j = 0; j <= i; ++j) fw[j * f + i] = Li[i * nsv + j];
    if (nbv > 0) {
      std::vector<double> G(size_t(nbv * nsv), 0.0);   // L21 * Linv, row-major nb x ns
      for (int64_t r = 0; r < nbv; ++r) {
        const double* l21 = Fm.data() + (nsv + r) * f;
        double* gr = G.data() + r * nsv;
        for (int64_t p = 0; p < nsv; ++p) {
          const double l = l21[p];
          if (l == 0.0) continue;
          const double* rp = Li.data() + p * nsv;
          for (int64_t j = 0; j <= p; ++j) gr[j] += l * rp[j];
        }
      }
      for (int64_t r = 0; r < nbv; ++r)
        for (int64_t j = 0; j < nsv; ++j) fw[j * f + nsv + r] = -G[r * nsv + j];
    }
    // Bw (column-major, ns x f): [Uinv | -Uinv U12]
    double* bw = F.bw.data() + F.bw_off[s];
    for (int64_t i = 0; i < nsv; ++i)
      for (int64_t j = i; j < nsv; ++j) bw[j * nsv + i] = Ui[i * nsv + j];
    if (nbv > 0) {
      std::vector<double> H(size_t(nsv * nbv), 0.0);   // Uinv * U12, row-major ns x nb
      for (int64_t i = 0; i < nsv; ++i) {
        double* hr = H.data() + i * nbv;
        for (int64_t p = i; p < nsv; ++p) {
          const double u = Ui[i * nsv + p];
          if (u == 0.0) continue;
          const double* u12 = Fm.data() + p * f + nsv;
          for (int64_t t = 0; t < nbv; ++t) hr[t] += u * u12[t];
        }
      }
      for (int64_t i = 0; i < nsv; ++i)
        for (int64_t t = 0; t < nbv; ++t) bw[(nsv + t) * nsv + i] = -H[i * nbv + t];
    }
    return -1;
  };

  for (int h = 0; h < F.nlev_fwd && bad < 0; ++h) {
    auto& L = by_height[h];
    if (int(L.size()) >= 2 * nthr) {
#pragma omp parallel for schedule(dynamic, 1)
      for (size_t t = 0; t < L.size(); ++t) {
        int r = factor_one(L[t], false);
        if (r >= 0) {
#pragma omp critical
          { bad = r; }
        }
      }
    } else {
      for (int s : L) {
        int r = factor_one(s, true);
        if (r >= 0) { bad = r; break; }
      }
    }
  }
  F.seconds_factor = secs(t1);
  if (bad >= 0) {
    *err = "nd_factor: zero or non-finite pivot at reordered index " + std::to_string(bad) +
           " (the preconditioner needs LU without pivoting)";
    return -4;
  }

  // assembly map of the forward fronts
  auto t2 = clk::now();
  const int64_t tot = F.front_off[S];
  F.asm_ptr.assign(tot + 1, 0);
  {
    std::vector<int32_t> pos(n, -1);
    std::vector<int64_t> tgt;   // per child row: target global front row
    std::vector<std::pair<int64_t, int64_t>> pairs;
    pairs.reserve(F.cb_off[S]);
    for (int s = 0; s < S; ++s) {
      const int64_t nsv = F.ns[s], nbv = F.nb[s];
      const int32_t a = F.j0[s];
      const int32_t* B = F.bnd.data() + F.bnd_off[s];
      for (int64_t p = 0; p < nsv; ++p) pos[a + p] = int32_t(p);
      for (int64_t p = 0; p < nbv; ++p) pos[B[p]] = int32_t(nsv + p);
      for (int c : children[s]) {
        const int32_t* Bc = F.bnd.data() + F.bnd_off[c];
        for (int64_t x = 0; x < F.nb[c]; ++x)
          pairs.emplace_back(F.front_off[s] + pos[Bc[x]], F.cb_off[c] + x);
      }
      for (int64_t p = 0; p < nsv; ++p) pos[a + p] = -1;
      for (int64_t p = 0; p < nbv; ++p) pos[B[p]] = -1;
    }
    std::sort(pairs.begin(), pairs.end());
    for (auto& pr : pairs) F.asm_ptr[pr.first + 1]++;
    for (int64_t i = 0; i < tot; ++i) F.asm_ptr[i + 1] += F.asm_ptr[i];
    F.asm_src.resize(pairs.size());
    for (size_t i = 0; i < pairs.size(); ++i) F.asm_src[i] = pairs[i].second;
  }
  F.seconds_post = secs(t2);
  return 0;
}

}  // namespace lrc
