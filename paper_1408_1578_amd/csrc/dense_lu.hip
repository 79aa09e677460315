// Dense LU with partial pivoting of floor(W) (Sec. 2.2) on the device, and
// the solves with its factors.
//
// floor(W) = E + antidiag(T) has one E entry per ordered pair of segments.
// When the segments are many (strongly curved boundaries) those entries
// couple the direction variables nearly all-to-all, every fill-reducing
// ordering leaves a dense Schur complement of a few thousand rows, and a
// sparse factorisation on the host takes minutes.  Such matrices are factored
// here instead, as dense complex matrices (N_W <= ~40000, 16 N_W^2 bytes of
// HBM), by the right-looking blocked algorithm with 64-column panels:
//   1. panel: for each column, pivot search (largest modulus, ties to the
//      lower row index; deterministic two-stage reduction), scaling, and
//      rank-1 update of the panel's later columns, in one launch per column;
//      the pivot rows stay where they are until the panel ends (rows chosen
//      so far are marked and left out), which is the same elimination with
//      the row swaps deferred;
//   2. the panel's row swaps (LAPACK's sequence, derived from the chosen
//      rows) applied to every column;
//   3. U12 = L11^{-1} A12 (one wave per column, L11 in LDS);
//   4. A22 -= L21 U12 on the FP64 matrix cores (v_mfma_f64_16x16x4, complex
//      products in the 3-multiplication form).
// Panels go in blocks of two or four: a panel's columns are updated by the
// block's earlier panels before it is factored, and the trailing matrix takes
// one update with K = 128 or 256 per block.
// After the factorisation the 256 x 256 diagonal blocks of L and U are
// inverted (with the same kernels); the solves apply the row permutation,
// then blocked forward and backward substitution made of matrix-core products
// only (diagonal block by its inverse, update of the remaining rows).  Matrices are column-major with leading
// dimension n; offsets are 64-bit.
#include <climits>
#include <vector>

#include "dense_lu.hpp"

namespace dp {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kNB = 64;       // panel width and solve block
// panels per block of the factorisation: 4 (trailing updates with K = 256)
// from n = kPanels4Min on, else 2 (K = 128).  Setup times with a dense
// floor(W), pairs against blocks of four: 37.5 / 38.8 ms at n = 3490, 90.5 /
// 90.5 at 6861, 318 / 294 at 13563 (the small products of a four-panel block
// cost more than the saved passes over a small trailing matrix).
constexpr int kPanels4Min = 8192;
constexpr int kParts = 1024;  // largest number of pivot-search partials

__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

__device__ __forceinline__ cplx crecip(cplx a) {
  const double d = cabs2(a);
  return d > 0.0 ? cplx{a.re / d, -a.im / d} : cplx{0.0, 0.0};
}

// (v, i) better than (bv, bi): larger modulus, ties to the smaller row
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// block (256 threads) reduction of (v, i) pairs; result in slot 0
__device__ __forceinline__ void reduce_best(double* sv, int* si) {
  const int t = threadIdx.x;
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s && better(sv[t + s], si[t + s], sv[t], si[t])) {
      sv[t] = sv[t + s];
      si[t] = si[t + s];
    }
    __syncthreads();
  }
}

// partials of max |A[r, c]|^2 over rows c..n-1
__global__ __launch_bounds__(256) void col_amax(const cplx* __restrict__ A, int n, int c, double* pv, int* pi) {
  __shared__ double sv[256];
  __shared__ int si[256];
  double bv = -1.0;
  int bi = INT_MAX;
  const size_t col = (size_t)c * n;
  for (int r = c + blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double v = cabs2(A[col + r]);
    if (better(v, r, bv, bi)) {
      bv = v;
      bi = r;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  reduce_best(sv, si);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

// Column c = k0 + j of the panel, in one launch.  Every block reduces the
// partials of column c (the same pivot row p in each: the largest modulus
// among the rows not yet chosen in this panel, ties to the lower row index),
// reads row p's panel entries, and updates its 64 rows among those not yet
// chosen: l = a/pivot in column c and the rank-1 update of the panel's later
// columns.  Wave w takes the later columns j + 1 + 16 w .. j + 16 (w + 1) of
// the block's rows, one row per lane, with every load before any store (one
// round trip; the matrix may alias, so loads after a store would wait for
// it); wave 0 also writes l and the partial of column c + 1 over its rows
// (when want_next) into the other partial buffer.  Row p is not moved:
// block 0 marks it (mark[p] = c; rows whose mark is below k0 are not chosen
// in this panel) and records it in plist[j].  A zero or non-finite pivot
// sets *info = c + 1 once and continues with 1/0 = 0.  A thread requests its
// first row's entries before the pivot is known (they do not depend on it),
// and the block's barriers order LDS only, so those loads run while the
// partials are reduced and the pivot row is read.
constexpr int kUpdChunk = 16;  // later columns per wave (4 waves cover the 63 of a panel)

// Block barrier for LDS only: the block's LDS accesses before it are complete,
// while its global loads may stay in flight across it (a full __syncthreads
// waits for those too).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// reduce_best with LDS-only barriers
__device__ __forceinline__ void reduce_best_lds(double* sv, int* si) {
  const int t = threadIdx.x;
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s && better(sv[t + s], si[t + s], sv[t], si[t])) {
      sv[t] = sv[t + s];
      si[t] = si[t + s];
    }
    lds_sync();
  }
}

__global__ __launch_bounds__(256) void panel_col(cplx* A, int n, int k0, int kb, int c, const double* pv_in,
                                                 const int* pi_in, int nparts, double* pv_out, int* pi_out,
                                                 int* mark, int* plist, int* info, int want_next) {
  __shared__ cplx prow[kNB];
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ int sp;
  const int j = c - k0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int j0 = j + 1 + kUpdChunk * w;                                  // this wave's first later column
  const int r0 = (w == 0 || j0 < kb) ? k0 + blockIdx.x * 64 + lane : n;  // waves without columns skip
  const int rstep = gridDim.x * 64;
  // this thread's first partial, then the first row's mark and entries,
  // requested before the pivot is known (they do not depend on it): loads
  // complete in order, so the partial comes first, and the row's entries
  // arrive while the partials are reduced
  // (straight-line, with the indices clamped to valid entries, so that the
  // wait for the partial does not have to assume the row's loads were skipped)
  const int q0 = tid < nparts ? tid : nparts - 1;  // nparts >= 1
  double bv = pv_in[q0];
  int bi = pi_in[q0];
  if (tid >= nparts) {
    bv = -1.0;
    bi = INT_MAX;
  }
  const int rr = r0 < n ? r0 : n - 1;
  const int mk0 = mark[rr];
  const cplx a0 = A[(size_t)c * n + rr];
  cplx x0[kUpdChunk];
#pragma unroll
  for (int u = 0; u < kUpdChunk; ++u) x0[u] = A[(size_t)(k0 + min(j0 + u, kb - 1)) * n + rr];
  for (int q = tid + 256; q < nparts; q += 256)
    if (better(pv_in[q], pi_in[q], bv, bi)) {
      bv = pv_in[q];
      bi = pi_in[q];
    }
  sv[tid] = bv;
  si[tid] = bi;
  lds_sync();
  reduce_best_lds(sv, si);
  const bool inrange = si[0] >= k0 && si[0] < n;
  const bool bad = !(sv[0] > 0.0) || !(sv[0] < 1e300) || !inrange;
  if (tid == 0) {
    int p = si[0];
    if (!inrange) {  // no finite candidate: the first row not yet chosen (one exists: n - c >= 1)
      p = k0;
      while (p < n - 1 && mark[p] >= k0) ++p;
    }
    sp = p;
  }
  lds_sync();
  const int p = sp;
  if (tid < kb) prow[tid] = A[(size_t)(k0 + tid) * n + p];
  lds_sync();
  const cplx inv = crecip(prow[j]);
  double nb = -1.0;
  int ni = INT_MAX;
  // l = a/pivot in column c (wave 0), the rank-1 update of this wave's
  // columns, and the candidate of column c + 1 (wave 0, its first column)
  auto row = [&](int r, const cplx a, cplx (&x)[kUpdChunk]) {
    const cplx l = cmul(a, inv);
    if (w == 0) A[(size_t)c * n + r] = l;
#pragma unroll
    for (int u = 0; u < kUpdChunk; ++u)
      if (j0 + u < kb) {
        const cplx v = prow[j0 + u];
        x[u] = {x[u].re - (l.re * v.re - l.im * v.im), x[u].im - (l.re * v.im + l.im * v.re)};
        A[(size_t)(k0 + j0 + u) * n + r] = x[u];
      }
    if (w == 0 && want_next) {
      const double v = cabs2(x[0]);
      if (better(v, r, nb, ni)) {
        nb = v;
        ni = r;
      }
    }
  };
  if (r0 < n && r0 != p && mk0 < k0) row(r0, a0, x0);
  for (int r = r0 + rstep; r < n; r += rstep) {  // more rows than 64 per block (n - k0 > 65536)
    if (r == p || mark[r] >= k0) continue;
    const cplx a = A[(size_t)c * n + r];
    cplx x[kUpdChunk];
#pragma unroll
    for (int u = 0; u < kUpdChunk; ++u)
      if (j0 + u < kb) x[u] = A[(size_t)(k0 + j0 + u) * n + r];
    row(r, a, x);
  }
  lds_sync();  // every thread is past its reads of the first reduction
  sv[tid] = nb;
  si[tid] = ni;
  lds_sync();
  reduce_best_lds(sv, si);
  if (tid == 0) {
    pv_out[blockIdx.x] = sv[0];
    pi_out[blockIdx.x] = si[0];
    if (blockIdx.x == 0) {
      mark[p] = c;
      plist[j] = p;
      if (bad && *info == 0) *info = c + 1;
    }
  }
}

// The panel's row swaps on every column (one thread per column).  LAPACK's
// sequence swaps row c = k0 + j with the row that holds plist[j] at step j,
// q_j = ipiv[c]: the chosen row is still at its own index unless that index
// is a position k0 + i filled at an earlier step i < j, which sent its row to
// q_i (so follow q_i, which lies beyond k0 + i, until it is not such a
// position).  Each block derives the sequence (thread 0, in LDS); block 0
// stores it in ipiv.
__global__ __launch_bounds__(256) void laswp(cplx* A, int n, int k0, int kb, const int* __restrict__ plist,
                                             int* ipiv) {
  __shared__ int q[kNB];
  if (threadIdx.x == 0) {
    for (int j = 0; j < kb; ++j) {
      int pos = plist[j];
      // each hop goes to a later step, so at most j hops
      for (int h = 0; h < j && pos >= k0 && pos < k0 + j; ++h) pos = q[pos - k0];
      q[j] = pos;
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < kb) ipiv[k0 + threadIdx.x] = q[threadIdx.x];
  for (int t = blockIdx.x * 256 + threadIdx.x; t < n; t += gridDim.x * 256) {
    const size_t col = (size_t)t * n;
    for (int j = 0; j < kb; ++j) {
      const int c = k0 + j, pr = q[j];
      if (pr != c) {
        const cplx a = A[col + c], b = A[col + pr];
        A[col + c] = b;
        A[col + pr] = a;
      }
    }
  }
}

// X = L^{-1} X for the unit lower kb x kb block L and kb x ncols X; one wave
// per column (lane = row), L in LDS.
__global__ __launch_bounds__(256) void trsm_lower_unit(const cplx* __restrict__ L, int ldl, cplx* X, int ldx, int kb,
                                                       int ncols) {
  __shared__ cplx Ls[kNB][kNB + 1];
  for (int e = threadIdx.x; e < kb * kb; e += 256) {
    const int r = e % kb, k = e / kb;
    Ls[r][k] = L[(size_t)k * ldl + r];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int col = blockIdx.x * 4 + (threadIdx.x >> 6); col < ncols; col += gridDim.x * 4) {
    cplx* x = X + (size_t)col * ldx;
    cplx v = lane < kb ? x[lane] : cplx{0.0, 0.0};
    for (int r = 0; r + 1 < kb; ++r) {
      const cplx xr = {__shfl(v.re, r), __shfl(v.im, r)};
      if (lane > r && lane < kb) {
        const cplx l = Ls[lane][r];
        v = {v.re - (l.re * xr.re - l.im * xr.im), v.im - (l.re * xr.im + l.im * xr.re)};
      }
    }
    if (lane < kb) x[lane] = v;
  }
}

// X = U^{-1} X for the upper kb x kb block U (non-unit diagonal).
__global__ __launch_bounds__(256) void trsm_upper(const cplx* __restrict__ U, int ldu, cplx* X, int ldx, int kb,
                                                  int ncols) {
  __shared__ cplx Us[kNB][kNB + 1];
  __shared__ cplx dinv[kNB];
  for (int e = threadIdx.x; e < kb * kb; e += 256) {
    const int r = e % kb, k = e / kb;
    Us[r][k] = U[(size_t)k * ldu + r];
  }
  __syncthreads();
  if (threadIdx.x < kb) dinv[threadIdx.x] = crecip(Us[threadIdx.x][threadIdx.x]);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int col = blockIdx.x * 4 + (threadIdx.x >> 6); col < ncols; col += gridDim.x * 4) {
    cplx* x = X + (size_t)col * ldx;
    cplx v = lane < kb ? x[lane] : cplx{0.0, 0.0};
    for (int r = kb - 1; r >= 0; --r) {
      if (lane == r) v = cmul(v, dinv[r]);
      const cplx xr = {__shfl(v.re, r), __shfl(v.im, r)};
      if (lane < r) {
        const cplx u = Us[lane][r];
        v = {v.re - (u.re * xr.re - u.im * xr.im), v.im - (u.re * xr.im + u.im * xr.re)};
      }
    }
    if (lane < kb) x[lane] = v;
  }
}

// C (M x N) -= A (M x K) B (K x N) (or C = -A B with overwrite), on the FP64
// matrix cores.
// Block: 4 waves, a 64 x 64 tile of C.  K runs in chunks of 16 through a
// double-buffered LDS stage, k-major (As[k][i], Bs[k][j]) so that the MFMA
// operands A[i][k] (lane i + 16k) and B[k][j] (lane j + 16k) are 16-element
// contiguous runs; each thread loads its 4 + 4 elements of the next chunk
// into registers before the current chunk's products and stores them after
// the barrier (67 KB of LDS: two blocks per CU).  Each wave owns a 32 x 32
// quarter (2 x 2 tiles of 16 x 16) with three accumulators per tile:
// T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi); C -= (T1 - T2) + i (T3 - T1 - T2).
// Result layout: register r of lane L holds row 4r + L/16, column L mod 16.
constexpr int kKC = 16;
__global__ __launch_bounds__(256) void zgemm_sub(const cplx* __restrict__ A, int lda, const cplx* __restrict__ B,
                                                 int ldb, cplx* C, int ldc, int M, int N, int K, int overwrite) {
  __shared__ cplx As[2][kKC][kNB + 1];
  __shared__ cplx Bs[2][kKC][kNB + 1];
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  // element q of a chunk (q = tid + 256 e, e < 4): A (i = q mod 64, k = q / 64),
  // B (k = q mod 16, j = q / 16)
  cplx ra[4], rb[4];
  auto load = [&](int kc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = tid + 256 * e;
      const int i = q & 63, ka = kc + (q >> 6);
      ra[e] = (m0 + i < M && ka < K) ? A[(size_t)ka * lda + m0 + i] : cplx{0.0, 0.0};
      const int kb = kc + (q & 15), j = q >> 4;
      rb[e] = (kb < K && n0 + j < N) ? B[(size_t)(n0 + j) * ldb + kb] : cplx{0.0, 0.0};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = tid + 256 * e;
      As[buf][q >> 6][q & 63] = ra[e];
      Bs[buf][q & 15][q >> 4] = rb[e];
    }
  };
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = 32 * (w & 1), j0 = 32 * (w >> 1);
  dbl4 T1[2][2], T2[2][2], T3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      T1[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
      T2[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
      T3[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  const int nch = (K + kKC - 1) / kKC;
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) load((ch + 1) * kKC);
#pragma unroll
    for (int s = 0; s < kKC / 4; ++s) {
      const int k = 4 * s + lk;
      cplx a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[buf][k][i0 + 16 * t + li];
        b[t] = Bs[buf][k][j0 + 16 * t + li];
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          T1[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].re, b[tb].re, T1[ta][tb], 0, 0, 0);
          T2[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].im, b[tb].im, T2[ta][tb], 0, 0, 0);
          T3[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].re + a[ta].im, b[tb].re + b[tb].im,
                                                            T3[ta][tb], 0, 0, 0);
        }
    }
    if (more) store(buf ^ 1);  // the other buffer was last read before the previous barrier
    __syncthreads();
  }
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + i0 + 16 * ta + 4 * r + lk;
        const int j = n0 + j0 + 16 * tb + li;
        if (i < M && j < N) {
          const double t1 = T1[ta][tb][r], t2 = T2[ta][tb][r], t3 = T3[ta][tb][r];
          cplx& c = C[(size_t)j * ldc + i];
          const cplx c0 = overwrite ? cplx{0.0, 0.0} : c;
          c = {c0.re - (t1 - t2), c0.im - (t3 - t1 - t2)};
        }
      }
}

// C (M x N) -= A (M x K) B (K x N), or C = -A B with overwrite, for the
// tall and skinny products of the triangular solves (N <= NB <= 16 columns,
// K <= 256): the matrix-core tile above would leave three quarters of its 64
// columns empty.  A block takes 16 rows and splits K into 16 groups: lane l of
// wave w takes row l mod 16 and group 4 w + l / 16, with the NB columns in
// registers, so that many blocks keep many short load chains in flight.  B's
// rows sit in LDS, each group's run offset by 4 elements so that the four
// groups of a wave read from different banks (within a group every lane reads
// the same element: a broadcast).  The groups are added in a fixed order:
// within the wave by lane exchanges, then over the waves through LDS.  Each
// element of A is read once.
template <int NB>
__global__ __launch_bounds__(256) void zgemm_ts(const cplx* __restrict__ A, int lda, const cplx* __restrict__ B,
                                                int ldb, cplx* C, int ldc, int M, int N, int K, int overwrite) {
  constexpr int kPad = 4;
  // B's rows, then (after the products) the partial sums [wave][column][row]
  __shared__ cplx Bs[256 * NB + 16 * kPad];
  cplx* red = Bs;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, kg = 4 * wv + (lane >> 4);
  const int i = blockIdx.x * 16 + r;
  const int kq = (K + 15) / 16;  // k per group
  // B along its columns (K NB <= 256 NB elements, NB per thread), all loads
  // issued before the first LDS store
  {
    cplx tb[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int j = e / K, k = e - j * K;
      tb[q] = e < K * NB && j < N ? B[(size_t)j * ldb + k] : cplx{0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < K * NB) {
        const int j = e / K, k = e - j * K;
        const int g = k / kq;
        Bs[g * (kq * NB + kPad) + (k - g * kq) * NB + j] = tb[q];
      }
    }
  }
  // this lane's (at most 16) elements of A, all loads in flight together
  const int k0 = kg * kq, nk = max(0, min(K, k0 + kq) - k0);
  cplx av[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) av[t] = t < nk && i < M ? A[(size_t)(k0 + t) * lda + i] : cplx{0.0, 0.0};
  __syncthreads();
  cplx acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = {0.0, 0.0};
  const cplx* bg = Bs + kg * (kq * NB + kPad);
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (t < nk) {
      const cplx* b = bg + t * NB;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const cplx bv = b[j];
        acc[j].re = fma(av[t].re, bv.re, fma(-av[t].im, bv.im, acc[j].re));
        acc[j].im = fma(av[t].re, bv.im, fma(av[t].im, bv.re, acc[j].im));
      }
    }
  }
  // the wave's four groups of this row: lanes l, l ^ 16, l ^ 32, l ^ 48
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    acc[j].re += __shfl_xor(acc[j].re, 16);
    acc[j].im += __shfl_xor(acc[j].im, 16);
    acc[j].re += __shfl_xor(acc[j].re, 32);
    acc[j].im += __shfl_xor(acc[j].im, 32);
  }
  __syncthreads();  // B is no longer read
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < NB; ++j) red[(wv * NB + j) * 16 + r] = acc[j];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 16 * NB; t += 256) {
    const int rr = t & 15, j = t >> 4;
    const int ii = blockIdx.x * 16 + rr;
    if (j < N && ii < M) {
      cplx v = red[j * 16 + rr];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        v.re += red[(w * NB + j) * 16 + rr].re;
        v.im += red[(w * NB + j) * 16 + rr].im;
      }
      cplx& c = C[(size_t)j * ldc + ii];
      const cplx c0 = overwrite ? cplx{0.0, 0.0} : c;
      c = {c0.re - v.re, c0.im - v.im};
    }
  }
}

__global__ void dense_scatter(cplx* A, int n, const int* __restrict__ rows, const int* __restrict__ cols,
                              const cplx* __restrict__ vals, int nnz) {
  for (int q = blockIdx.x * 256 + threadIdx.x; q < nnz; q += gridDim.x * 256)
    A[(size_t)cols[q] * n + rows[q]] = vals[q];
}

__global__ void gather_perm(const cplx* __restrict__ z, cplx* t, const int* __restrict__ perm, int n, int nrhs) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = idx % n;
    const size_t c = idx / n;
    t[idx] = z[c * n + perm[i]];
  }
}

int nblocks(int64_t rows, int cap) {
  int64_t g = (rows + 255) / 256;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

void launch_gemm_sub(hipStream_t st, const cplx* A, int lda, const cplx* B, int ldb, cplx* C, int ldc, int M, int N,
                     int K, int overwrite = 0) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  if (N <= 16 && K <= 256) {
    const int g = (M + 15) / 16;
    if (N <= 4) zgemm_ts<4><<<g, 256, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, overwrite);
    else if (N <= 8) zgemm_ts<8><<<g, 256, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, overwrite);
    else zgemm_ts<16><<<g, 256, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, overwrite);
    return;
  }
  dim3 grid((M + 63) / 64, (N + 63) / 64);
  zgemm_sub<<<grid, 256, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, overwrite);
}

// X (ld x ld) = identity on its first kb rows and columns, zero elsewhere
__global__ void set_identity(cplx* X, int ld, int kb) {
  const size_t tot = (size_t)ld * ld;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int r = idx % ld, c = idx / ld;
    X[idx] = (r == c && r < kb) ? cplx{1.0, 0.0} : cplx{0.0, 0.0};
  }
}

__global__ void negate(cplx* X, size_t tot) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x)
    X[idx] = {-X[idx].re, -X[idx].im};
}

}  // namespace

int DenseLU::assemble(hipStream_t st, int n_, const std::vector<int>& rows, const std::vector<int>& cols,
                      const std::vector<cplx>& vals) {
  n = n_;
  const size_t bytes = (size_t)n * n * sizeof(cplx);
  DP_TRY(a.reserve(bytes));
  DP_HIP(hipMemsetAsync(a.p, 0, bytes, st));
  DevBuf dr, dc, dv;
  DP_TRY(dr.reserve(std::max<size_t>(1, rows.size()) * sizeof(int)));
  DP_TRY(dc.reserve(std::max<size_t>(1, cols.size()) * sizeof(int)));
  DP_TRY(dv.reserve(std::max<size_t>(1, vals.size()) * sizeof(cplx)));
  const int nnz = (int)vals.size();
  if (nnz > 0) {
    DP_HIP(hipMemcpyAsync(dr.p, rows.data(), nnz * sizeof(int), hipMemcpyHostToDevice, st));
    DP_HIP(hipMemcpyAsync(dc.p, cols.data(), nnz * sizeof(int), hipMemcpyHostToDevice, st));
    DP_HIP(hipMemcpyAsync(dv.p, vals.data(), nnz * sizeof(cplx), hipMemcpyHostToDevice, st));
    dense_scatter<<<nblocks(nnz, 4096), 256, 0, st>>>(a.as<cplx>(), n, dr.as<int>(), dc.as<int>(), dv.as<cplx>(),
                                                      nnz);
    DP_HIP(hipGetLastError());
  }
  DP_HIP(hipStreamSynchronize(st));
  dr.release();
  dc.release();
  dv.release();
  return DP_OK;
}

int DenseLU::factor(hipStream_t st) {
  cplx* A = a.as<cplx>();
  DP_TRY(ipiv.reserve((size_t)n * sizeof(int)));
  // two partial buffers (kParts doubles, kParts ints each), the singularity
  // flag, the panel's chosen rows and the row marks
  const size_t wbytes = 2 * kParts * (sizeof(double) + sizeof(int)) + (1 + kNB + (size_t)n) * sizeof(int);
  DP_TRY(work.reserve(wbytes));
  double* pvb[2] = {work.as<double>(), work.as<double>() + kParts};
  int* pib[2] = {reinterpret_cast<int*>(pvb[1] + kParts), reinterpret_cast<int*>(pvb[1] + kParts) + kParts};
  int* info = pib[1] + kParts;
  int* plist = info + 1;
  int* mark = plist + kNB;
  DP_HIP(hipMemsetAsync(info, 0, sizeof(int), st));
  DP_HIP(hipMemsetAsync(mark, 0xFF, (size_t)n * sizeof(int), st));  // -1: never chosen
  int* ip = ipiv.as<int>();
  // one 64-column panel: pivots and eliminations, then its row swaps on
  // every column
  auto panel = [&](int k0, int kb) {
    const int parts = (int)std::min<int64_t>(kParts, ((int64_t)n - k0 + 63) / 64);  // 64 rows per panel_col block
    col_amax<<<parts, 256, 0, st>>>(A, n, k0, pvb[0], pib[0]);
    for (int j = 0; j < kb; ++j)
      panel_col<<<parts, 256, 0, st>>>(A, n, k0, kb, k0 + j, pvb[j & 1], pib[j & 1], parts, pvb[(j + 1) & 1],
                                       pib[(j + 1) & 1], mark, plist, info, j + 1 < kb ? 1 : 0);
    laswp<<<nblocks(n, 4096), 256, 0, st>>>(A, n, k0, kb, plist, ip);
  };
  // X = L^{-1} X for the unit lower block of the panel at k0 (kb x kb) and the
  // kb x ncols block of rows k0.. and columns c0..
  auto trsm = [&](int k0, int kb, int c0, int ncols) {
    trsm_lower_unit<<<std::min(1024, (ncols + 3) / 4), 256, 0, st>>>(A + (size_t)k0 * n + k0, n,
                                                                      A + (size_t)c0 * n + k0, n, kb, ncols);
  };
  // U rows of the first np_ panels of the block at K0 (all 64 wide) on the
  // columns c0..c0 + nc - 1: block forward substitution, panel by panel
  auto bsub = [&](int K0, int np_, int c0, int nc) {
    for (int h = 0; h < np_; ++h) {
      const int off = K0 + h * kNB;
      trsm(off, kNB, c0, nc);
      const int below = (np_ - 1 - h) * kNB;
      if (below > 0)
        launch_gemm_sub(st, A + (size_t)off * n + off + kNB, n, A + (size_t)c0 * n + off, n,
                        A + (size_t)c0 * n + off + kNB, n, below, nc, kNB);
    }
  };
  // Blocks of kPanels panels.  Before a panel is factored, its columns take
  // the block's earlier panels: their U rows by block forward substitution,
  // then one update of the rows below with K = 64 (earlier panels).  After
  // the block, the trailing columns take the U rows of all its panels and one
  // update with K = 64 kPanels: a half or a quarter of the passes over the
  // trailing matrix of one update per panel.
  const int kPanels = n >= kPanels4Min ? 4 : 2;
  for (int K0 = 0; K0 < n; K0 += kPanels * kNB) {
    const int KB = std::min(kPanels * kNB, n - K0);
    int np_ = 0;
    for (int c = K0; c < K0 + KB; c += kNB, ++np_) {
      const int w = std::min(kNB, K0 + KB - c);
      if (np_ > 0) {
        bsub(K0, np_, c, w);
        launch_gemm_sub(st, A + (size_t)K0 * n + c, n, A + (size_t)c * n + K0, n, A + (size_t)c * n + c, n, n - c,
                        w, c - K0);
      }
      panel(c, w);
    }
    const int rest = n - K0 - KB;
    if (rest > 0) {  // the block's panels are all full
      bsub(K0, np_, K0 + KB, rest);
      launch_gemm_sub(st, A + (size_t)K0 * n + K0 + KB, n, A + (size_t)(K0 + KB) * n + K0, n,
                      A + (size_t)(K0 + KB) * n + K0 + KB, n, rest, rest, KB);
    }
    DP_HIP(hipGetLastError());
  }
  // permutation of the row swaps: (P z)[i] = z[perm[i]]
  std::vector<int> h(n), pm(n);
  int hinfo = 0;
  DP_HIP(hipMemcpyAsync(h.data(), ip, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
  DP_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  if (hinfo != 0) {
    set_error("dense LU of floor(W): zero pivot in column %d", hinfo - 1);
    return DP_ESINGULAR;
  }
  for (int i = 0; i < n; ++i) pm[i] = i;
  for (int c = 0; c < n; ++c) std::swap(pm[c], pm[h[c]]);
  DP_TRY(perm.reserve((size_t)n * sizeof(int)));
  DP_HIP(hipMemcpyAsync(perm.p, pm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
  DP_HIP(hipStreamSynchronize(st));
  return block_inverses(st);
}

// -L_bb^{-1} and -U_bb^{-1} for every kSB x kSB diagonal block (the last one
// may be smaller), by blocked substitution on identity columns with the
// factorisation's own kernels; stored column-major with leading dimension kSB.
int DenseLU::block_inverses(hipStream_t st) {
  const cplx* A = a.as<cplx>();
  nsb = (n + kSB - 1) / kSB;
  const size_t per = (size_t)kSB * kSB;
  DP_TRY(dinvL.reserve(nsb * per * sizeof(cplx)));
  DP_TRY(dinvU.reserve(nsb * per * sizeof(cplx)));
  for (int bk = 0; bk < nsb; ++bk) {
    const int b0 = bk * kSB, kb = std::min(kSB, n - b0);
    cplx* XL = dinvL.as<cplx>() + bk * per;
    cplx* XU = dinvU.as<cplx>() + bk * per;
    set_identity<<<nblocks((int64_t)per, 1024), 256, 0, st>>>(XL, kSB, kb);
    set_identity<<<nblocks((int64_t)per, 1024), 256, 0, st>>>(XU, kSB, kb);
    for (int s0 = 0; s0 < kb; s0 += kNB) {
      const int sk = std::min(kNB, kb - s0);
      trsm_lower_unit<<<std::min(1024, (kb + 3) / 4), 256, 0, st>>>(A + (size_t)(b0 + s0) * n + b0 + s0, n, XL + s0,
                                                                    kSB, sk, kb);
      launch_gemm_sub(st, A + (size_t)(b0 + s0) * n + b0 + s0 + sk, n, XL + s0, kSB, XL + s0 + sk, kSB,
                      kb - s0 - sk, kb, sk);
    }
    for (int s0 = ((kb - 1) / kNB) * kNB; s0 >= 0; s0 -= kNB) {
      const int sk = std::min(kNB, kb - s0);
      trsm_upper<<<std::min(1024, (kb + 3) / 4), 256, 0, st>>>(A + (size_t)(b0 + s0) * n + b0 + s0, n, XU + s0, kSB,
                                                               sk, kb);
      launch_gemm_sub(st, A + (size_t)(b0 + s0) * n + b0, n, XU + s0, kSB, XU, kSB, s0, kb, sk);
    }
    negate<<<nblocks((int64_t)per, 1024), 256, 0, st>>>(XL, per);
    negate<<<nblocks((int64_t)per, 1024), 256, 0, st>>>(XU, per);
  }
  DP_HIP(hipGetLastError());
  DP_HIP(hipStreamSynchronize(st));
  return DP_OK;
}

// u = A^{-1} z: t = P z; forward over kSB-row blocks, y_b = L_bb^{-1} t_b
// (a matrix-core product with the stored inverse) and t_below -= L_below,b y_b;
// backward, u_b = U_bb^{-1} y_b and y_above -= U_above,b u_b.  Each step is two
// matrix-core launches; t and y are workspaces, so no product reads what
// another writes.
int DenseLU::solve(hipStream_t st, const cplx* z, cplx* u, int nrhs) {
  const size_t bytes = (size_t)n * nrhs * sizeof(cplx);
  DP_TRY(tws.reserve(bytes));
  DP_TRY(yws.reserve(bytes));
  return solve_ws(st, z, u, nrhs, tws.as<cplx>(), yws.as<cplx>());
}

int DenseLU::solve_ws(hipStream_t st, const cplx* z, cplx* u, int nrhs, cplx* t, cplx* y) const {
  const cplx* A = a.as<cplx>();
  const size_t per = (size_t)kSB * kSB;
  gather_perm<<<nblocks((int64_t)n * nrhs, 8192), 256, 0, st>>>(z, t, perm.as<int>(), n, nrhs);
  for (int bk = 0; bk < nsb; ++bk) {
    const int b0 = bk * kSB, kb = std::min(kSB, n - b0);
    launch_gemm_sub(st, dinvL.as<cplx>() + bk * per, kSB, t + b0, n, y + b0, n, kb, nrhs, kb, 1);
    launch_gemm_sub(st, A + (size_t)b0 * n + b0 + kb, n, y + b0, n, t + b0 + kb, n, n - b0 - kb, nrhs, kb);
  }
  for (int bk = nsb - 1; bk >= 0; --bk) {
    const int b0 = bk * kSB, kb = std::min(kSB, n - b0);
    launch_gemm_sub(st, dinvU.as<cplx>() + bk * per, kSB, y + b0, n, u + b0, n, kb, nrhs, kb, 1);
    launch_gemm_sub(st, A + (size_t)b0 * n, n, u + b0, n, y, n, b0, nrhs, kb);
  }
  DP_HIP(hipGetLastError());
  return DP_OK;
}

void DenseLU::release() {
  a.release();
  dinvL.release();
  dinvU.release();
  tws.release();
  yws.release();
  ipiv.release();
  perm.release();
  work.release();
  n = 0;
}

}  // namespace dp
