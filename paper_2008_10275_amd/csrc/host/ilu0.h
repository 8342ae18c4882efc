// Incomplete LU without fill (ILU(0)) of a sparse matrix, and the level sets
// of its triangular solves (host code, compiled without HIP).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "ndfact.h"

namespace lrc {

// L (unit lower) and U (upper with diagonal) on the pattern of A, stored in
// A's CSR layout: entries left of the diagonal hold L, the rest U.
struct Ilu0 {
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> lu;
  std::vector<int32_t> diag;        // position of the diagonal entry of each row
  // rows grouped by level: forward (L) and backward (U) solves; level l holds
  // rows_f[off_f[l] .. off_f[l + 1])
  std::vector<int32_t> rows_f, rows_b;
  std::vector<int32_t> off_f, off_b;
};

// Returns 0, -4 for a zero or non-finite pivot (err says which row), -1 for a
// missing diagonal entry or an unsorted row.
int ilu0_factor(const CsrHost& A, Ilu0* out, std::string* err);

}  // namespace lrc
