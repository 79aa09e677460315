// Host sparse LU of floor(W) with level schedules for the device solves.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace dp {

struct SparseLU {
  int n = 0;
  // W u = z  <=>  zp[k] = z[perm_in[k]];  L y = zp;  U u' = y;  u[perm_out[b]] = u'[b]
  std::vector<int> perm_in, perm_out;
  std::vector<int> Lp, Lj;  // CSR, strictly lower part of the unit lower factor
  std::vector<std::complex<double>> Lx;
  std::vector<int> Up, Uj;  // CSR, strictly upper part of U
  std::vector<std::complex<double>> Ux, Ud;  // Ud: diagonal of U
  std::vector<int> lvlL_ptr, lvlL_rows, lvlU_ptr, lvlU_rows;
};

// W given in CSC (colptr, rowind, values), n x n.  Returns DP_OK,
// DP_ESINGULAR, or kSparseFillLimit when nnz(L + U) would exceed max_fill
// (predicted from the ordering) or twice it (in the numeric factorisation).
constexpr int kSparseFillLimit = 2;
int sparse_lu_factor(int n, const std::vector<int>& colptr, const std::vector<int>& rowind,
                     const std::vector<std::complex<double>>& val, SparseLU& out,
                     int64_t max_fill = INT64_MAX);

// The two halves of sparse_lu_factor.  The ordering needs only the pattern
// (so it can run before the values are known); it is empty when the
// predicted fill exceeds max_fill.  The numeric factorisation takes that
// ordering and returns DP_OK, DP_ESINGULAR or kSparseFillLimit (fill beyond
// twice max_fill).
std::vector<int> sparse_lu_order(int n, const std::vector<int>& colptr, const std::vector<int>& rowind,
                                 int64_t max_fill);
int sparse_lu_factor_ordered(int n, const std::vector<int>& colptr, const std::vector<int>& rowind,
                             const std::vector<std::complex<double>>& val, const std::vector<int>& order,
                             SparseLU& out, int64_t max_fill = INT64_MAX);

}  // namespace dp
