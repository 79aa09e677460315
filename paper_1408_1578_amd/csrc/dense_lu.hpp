// Dense LU with partial pivoting of floor(W) on the device (dense_lu.hip).
#pragma once

#include <vector>

#include "dp_internal.hpp"

namespace dp {

struct DenseLU {
  int n = 0;
  DevBuf a;     // n x n column-major: unit lower L below the diagonal, U on and above
  DevBuf ipiv;  // row swapped with row c at step c
  DevBuf perm;  // (P z)[i] = z[perm[i]]
  DevBuf work;  // pivot-search partials (two buffers), singularity flag, a panel's pivot rows, row marks
  static constexpr int kSB = 256;  // block size of the solves
  int nsb = 0;                     // diagonal blocks
  DevBuf dinvL, dinvU;  // -(L_bb)^{-1}, -(U_bb)^{-1} per diagonal block (kSB x kSB, column-major)
  DevBuf tws, yws;      // solve workspaces (n x nrhs)
  // zero n x n matrix with the given (row, col, value) entries (no duplicates)
  int assemble(hipStream_t st, int n, const std::vector<int>& rows, const std::vector<int>& cols,
               const std::vector<cplx>& vals);
  // P A = L U in place, then the inverses of the diagonal blocks; DP_ESINGULAR
  // on a zero pivot column
  int factor(hipStream_t st);
  int block_inverses(hipStream_t st);
  // u = A^{-1} z for nrhs columns (n x nrhs column-major, z and u distinct),
  // with the workspaces tws / yws (grown here as needed)
  int solve(hipStream_t st, const cplx* z, cplx* u, int nrhs);
  // the same with caller-provided workspaces t and y (n x nrhs each): kernel
  // launches only, no allocation
  int solve_ws(hipStream_t st, const cplx* z, cplx* u, int nrhs, cplx* t, cplx* y) const;
  void release();
};

}  // namespace dp
