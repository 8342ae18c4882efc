// ILU(0): the LU factorisation restricted to the sparsity pattern of A (the
// standard incomplete factorisation with no fill, row by row in IKJ order):
// for row i and each k < i in its pattern, in increasing order,
//   a_ik <- a_ik / a_kk,   a_ij <- a_ij - a_ik a_kj  for j > k in both patterns.
// The forward levels put row i one level after the latest row its L part
// reads; the backward levels likewise for U (rows in decreasing order).
#include "ilu0.h"

#include <algorithm>
#include <cmath>

namespace lrc {

int ilu0_factor(const CsrHost& A, Ilu0* out, std::string* err) {
  const int64_t n = A.n;
  Ilu0& F = *out;
  F.n = n;
  F.rowptr = A.rowptr;
  F.col = A.col;
  F.lu = A.val;
  F.diag.assign(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
      if (e > A.rowptr[i] && A.col[e] <= A.col[e - 1]) {
        if (err) *err = "ilu0: columns of row " + std::to_string(i) + " are not ascending";
        return -1;
      }
      if (A.col[e] == i) F.diag[i] = int32_t(e);
    }
    if (F.diag[i] < 0) {
      if (err) *err = "ilu0: row " + std::to_string(i) + " has no diagonal entry";
      return -1;
    }
  }
  std::vector<int64_t> pos(n, -1);   // column -> position in the current row
  for (int64_t i = 0; i < n; ++i) {
    const int64_t b = F.rowptr[i], e1 = F.rowptr[i + 1];
    for (int64_t e = b; e < e1; ++e) pos[F.col[e]] = e;
    for (int64_t e = b; e < e1 && F.col[e] < i; ++e) {
      const int32_t k = F.col[e];
      const double piv = F.lu[F.diag[k]];
      F.lu[e] /= piv;
      const double lik = F.lu[e];
      for (int64_t f = F.diag[k] + 1; f < F.rowptr[k + 1]; ++f) {
        const int64_t p = pos[F.col[f]];
        if (p >= 0) F.lu[p] -= lik * F.lu[f];
      }
    }
    for (int64_t e = b; e < e1; ++e) pos[F.col[e]] = -1;
    const double d = F.lu[F.diag[i]];
    if (!(std::isfinite(d) && d != 0.0)) {
      if (err) *err = "ilu0: zero or non-finite pivot at row " + std::to_string(i);
      return -4;
    }
  }
  // level sets
  std::vector<int32_t> lf(n, 0), lb(n, 0);
  int32_t nf = 0, nb = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t l = 0;
    for (int64_t e = F.rowptr[i]; e < F.diag[i]; ++e) l = std::max(l, lf[F.col[e]] + 1);
    lf[i] = l;
    nf = std::max(nf, l + 1);
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    int32_t l = 0;
    for (int64_t e = F.diag[i] + 1; e < F.rowptr[i + 1]; ++e) l = std::max(l, lb[F.col[e]] + 1);
    lb[i] = l;
    nb = std::max(nb, l + 1);
  }
  auto group = [&](const std::vector<int32_t>& lev, int32_t nl, std::vector<int32_t>& rows,
                   std::vector<int32_t>& off) {
    off.assign(nl + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++off[lev[i] + 1];
    for (int32_t l = 0; l < nl; ++l) off[l + 1] += off[l];
    rows.assign(n, 0);
    std::vector<int32_t> at(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[at[lev[i]]++] = int32_t(i);
  };
  group(lf, nf, F.rows_f, F.off_f);
  group(lb, nb, F.rows_b, F.off_b);
  return 0;
}

}  // namespace lrc
