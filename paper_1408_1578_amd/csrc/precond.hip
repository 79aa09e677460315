// Directional preconditioner of Sec. 2 on the GPU.
//
// Setup (dp_precond_build), in the paper's order:
//   Sec. 2.1  segments P_1..P_m (host, O(m)); per segment size class s:
//             the flat block B_s (Kress-discretised operator on a straight
//             segment of s points), B_s^{-1} (Gauss-Jordan, partial
//             pivoting), the partial Fourier factor
//             U_s(a, j) = exp(2 pi i j (a - (s-1)/2)/s), j = -J..J (eq. (12)),
//             S_s = U_s^t B_s^{-1} U_s, T_s = S_s^{-1} (Sec. 2.2) and its
//             thresholded floor(T_s);
//             centres c_i, tangents t_i and m_c first-kind Chebyshev points of
//             every segment by trigonometric interpolation of the nodes;
//             for every ordered pair i != j: the rounded directions
//             k^i_ij = [omega a_ij . t_i]_i, k^j_ij = [-omega a_ij . t_j]_j and
//             e_ij = alpha_i^t M~_ij(R_i, R_j) alpha_j (eq. (14)), one block
//             per pair.
//   Sec. 2.2  floor(W) = E + antidiag(T) assembled and LU-factored on the
//             host (sparse, see sparse_lu.cpp); factors copied to the device.
// Apply (eq. (19) on (v, 0, 0)), all on the device:
//   y = B^{-1} v; g = U^t y; z = floor(T) g; u = floor(W)^{-1} z;
//   h = z - floor(T) u; q = y - B^{-1} (U h).
// The per-segment dense products are batched complex GEMMs whose left operand
// is shared by all segments of a size class.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <map>
#include <system_error>
#include <thread>
#include <mutex>
#include <queue>
#include <vector>

#include "dp_internal.hpp"
#include "dense_lu.hpp"
#include "sparse_lu.hpp"

namespace dp {

using zc = std::complex<double>;
constexpr double kInv4Pi_p = 0.079577471545947667884441881686257181;

struct SizeClass {
  int s = 0, J = 0, K = 0;
  DevBuf Binv, U, Ut, Tt, alpha;
  DevBuf Binv32, U32, Ut32, Tt32;  // single-precision copies (mixed-precision apply)
  std::vector<cplx> T;  // full T_s on the host (antidiagonal goes into floor(W))
};

struct Precond {
  int m = 0, NW = 0, m_c = 10;
  std::vector<int> off, len, cls, J, offK;
  std::vector<SizeClass> classes;
  DevBuf d_segs;    // int4 per segment: off, len, offK, cls
  DevBuf d_ptrs;    // per class: Binv, U, Ut, Tt pointers
  DevBuf d_ptrs32;  // the same for the single-precision copies
  DevBuf d_dims;    // per class: s, K
  // E
  std::vector<int> eidx;  // 4 per pair
  std::vector<cplx> eval;
  // sparse LU on the device
  SparseLU lu;
  DevBuf Lp, Lj, Lx, Up, Uj, Ux, Ud, lvlL, lvlLr, lvlU, lvlUr, pin, pout;
  int nlevL = 0, nlevU = 0;
  // step streams of the single-wave LDS-resident solve (L then U), FP64 and FP32
  DevBuf slots, slots32;
  int nsteps = 0;
  bool lds_solve = false, lds_solve32 = false;
  // dense device LU of floor(W) (when the sparse factors would fill in)
  bool dense_w = false;
  DenseLU dlu;
  int64_t nnzW = 0;
  DevBuf wy, wg, wz, wu, wt, wn;  // apply workspaces
  DevBuf sy, sg, sz, su, sn, sv, sq;  // single-precision apply workspaces
  // graph of the apply (input win, output wq), captured for g_nrhs columns
  bool graphs = true;
  hipGraphExec_t gexec = nullptr;
  int g_nrhs = -1, g_calls = 0;
  DevBuf win, wq;
  // the same for the single-precision apply
  bool graphs32 = true;
  hipGraphExec_t gexec32 = nullptr;
  int g32_nrhs = -1, g32_calls = 0;
  std::vector<void*> g_sig, g32_sig;  // workspace addresses each graph was captured with
  double t_setup = 0;
};

// ------------------------------------------------------------------ helpers
static int grid1(size_t tot) {
  size_t g = (tot + 255) / 256;
  return (int)(g > 8192 ? 8192 : (g ? g : 1));
}

template <class T>
static int upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  DP_TRY(b.reserve(std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) DP_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return DP_OK;
}

__device__ __forceinline__ double round_half_away(double x) { return x >= 0 ? floor(x + 0.5) : -floor(-x + 0.5); }

// ------------------------------------------------------------------ flat blocks
// Row B(d), d = 0..s-1 of the symmetric Toeplitz flat block (spacing ds,
// parameter speed sp = L/(2 pi), global Kress table C with C[0] = R_0).
//   soft: B = 1/2 - i eta S_flat,
//     S_flat(d) = ds (i/4) H0(omega d ds) - C_d sp J0/(4 pi)           (d >= 1)
//     S_flat(0) = -R_0 sp/(4 pi) + dt sp (i/4 - gamma/(2 pi) - log(omega sp/2)/(2 pi))
//   hard: B = 1/2 + N_flat/(i eta), N_flat = f.p. (i omega/4) H1(omega r)/r:
//     N_flat(d) = ds (i omega/4) H1(omega r)/r - C_d sp (omega/(4 pi)) J1(omega r)/r
//                 + [d = 1] 1/(4 pi ds)                               (r = d ds)
//     N_flat(0) = R_0 k1 + dt k2 - pi/(6 ds) - 1/(2 pi ds),
//       k1 = -(omega^2/(8 pi)) sp,
//       k2 = sp (i omega^2/8 - (omega^2/(4 pi)) (log(omega sp/2) + gamma - 1/2))
//   (Laplace part 1/(2 pi r^2) by the finite-part trapezoid correction; the
//   log-singular remainder by the Kress rule.)
__global__ void flat_row(const double* __restrict__ C, cplx* row, int s, int n, double L, double omega,
                         double eta, int kind) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= s) return;
  const double ds = L / n, sp = L / (2.0 * kPi), dt = 2.0 * kPi / n;
  cplx v;
  if (kind == DP_SOFT) {
    cplx S;
    if (d == 0) {
      S = {-C[0] * sp * kInv4Pi_p + dt * sp * (-kEulerGamma - log(0.5 * omega * sp)) * (2.0 * kInv4Pi_p),
           0.25 * dt * sp};
    } else {
      const H01 h = hankel01(omega * d * ds);
      S = {-0.25 * ds * h.h0.im - C[d] * sp * kInv4Pi_p * h.h0.re, 0.25 * ds * h.h0.re};
    }
    v = {eta * S.im, -eta * S.re};  // -i eta S
  } else {
    cplx N;
    if (d == 0) {
      const double k1 = -(omega * omega / 8.0 / kPi) * sp;
      const double k2re = -sp * (omega * omega * kInv4Pi_p) * (log(0.5 * omega * sp) + kEulerGamma - 0.5);
      const double k2im = sp * omega * omega / 8.0;
      N = {C[0] * k1 + dt * k2re - kPi / (6.0 * ds) - 1.0 / (2.0 * kPi * ds), dt * k2im};
    } else {
      const double r = d * ds;
      const H01 h = hankel01(omega * r);
      // (i omega/4) H1 / r * ds
      N = {-0.25 * omega * h.h1.im / r * ds - C[d] * sp * omega * kInv4Pi_p * h.h1.re / r,
           0.25 * omega * h.h1.re / r * ds};
      if (d == 1) N.re += 1.0 / (4.0 * kPi * ds);
    }
    v = {N.im / eta, -N.re / eta};  // N/(i eta) = -i N/eta
  }
  if (d == 0) v.re += 0.5;
  row[d] = v;
}

// Dense s x s Toeplitz matrix from its first row, augmented with the identity
// (row-major s x 2s) for Gauss-Jordan.
__global__ void toeplitz_aug(const cplx* __restrict__ row, cplx* A, int s) {
  const size_t tot = (size_t)s * 2 * s;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = idx / (2 * s), c = idx % (2 * s);
    A[idx] = c < s ? row[abs(r - c)] : cplx{(c - s == r) ? 1.0 : 0.0, 0.0};
  }
}

__global__ void copy_right_half(const cplx* __restrict__ A, cplx* out, int s) {
  const size_t tot = (size_t)s * s;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = idx / s, c = idx % s;
    out[idx] = A[(size_t)r * 2 * s + s + c];
  }
}

// ------------------------------------------------------------ batched Gauss-Jordan
// Several augmented row-major s x 2s matrices [M | I] inverted together, one
// launch per elimination step k for all of them.  Step k reads buffer k % 2
// and writes buffer (k + 1) % 2, so no block sees another's partial update:
// the pivot row p (largest |A[i][k]| over rows i >= k, lowest index on ties,
// found by every block alike) becomes row k scaled by 1/A[p][k], the old row
// k moves to row p, and every other row loses its column-k multiple of the
// new row k.  Column k itself is not written (no later step reads it); the
// new column k + 1 is also kept contiguously for the next pivot search and
// multipliers.  After s steps the right half of buffer s % 2 is M^{-1}.  A zero pivot column sets
// status[matrix].
struct GJMat {
  cplx* a[2];
  cplx* col[2];  // contiguous copies of the pivot column of buffer k % 2 (column k)
  int s;
  int res;       // set by gj_invert: the buffer a[res] that holds the result
};
struct GJBatch {
  GJMat m[8];
  int* status;
};

__global__ __launch_bounds__(256) void gj_step(GJBatch b, int k) {
  const GJMat M = b.m[blockIdx.y];
  const int s = M.s;
  const int i = blockIdx.x;  // this block's row
  if (k >= s || i >= s) return;
  const int w = 2 * s;
  const cplx* A = M.a[k & 1];
  cplx* O = M.a[(k + 1) & 1];
  const cplx* colk = M.col[k & 1];
  cplx* coln = M.col[(k + 1) & 1];
  // pivot: wave-level argmax (ties to the lower row), then across the 4 waves
  __shared__ double bv[4];
  __shared__ int bi[4];
  double best = -1.0;
  int bidx = s;
  for (int i = k + threadIdx.x; i < s; i += 256) {
    const cplx a = colk[i];
    const double m = a.re * a.re + a.im * a.im;
    if (m > best) {
      best = m;
      bidx = i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(best, off);
    const int oi = __shfl_xor(bidx, off);
    if (o > best || (o == best && oi < bidx)) {
      best = o;
      bidx = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    bv[threadIdx.x >> 6] = best;
    bi[threadIdx.x >> 6] = bidx;
  }
  __syncthreads();
  best = bv[0];
  int p = bi[0];
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (bv[q] > best || (bv[q] == best && bi[q] < p)) {
      best = bv[q];
      p = bi[q];
    }
  if (!(best > 0.0)) {
    if (i == 0 && threadIdx.x == 0) b.status[blockIdx.y] = 1;
    return;
  }
  const cplx pv = colk[p];
  const double den = pv.re * pv.re + pv.im * pv.im;
  const cplx inv = {pv.re / den, -pv.im / den};
  // row i, columns k + 1 .. 2s - 1, four per thread in flight
  const int src = (i == p) ? k : i;
  const cplx m = colk[src];
  const cplx* prow = A + (size_t)p * w;
  const cplx* srow = A + (size_t)src * w;
  cplx* orow = O + (size_t)i * w;
  for (int c0 = k + 1 + threadIdx.x; c0 < w; c0 += 1024) {
    cplx pa[4], sa[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = min(c0 + 256 * u, w - 1);
      pa[u] = prow[c];
      sa[u] = srow[c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + 256 * u;
      if (c < w) {
        const cplx pr = cmul(pa[u], inv);
        cplx v = pr;
        if (i != k)
          v = {sa[u].re - (m.re * pr.re - m.im * pr.im), sa[u].im - (m.re * pr.im + m.im * pr.re)};
        orow[c] = v;
        if (c == k + 1) coln[i] = v;
      }
    }
  }
}

// Gauss–Jordan steps k .. k + nb - 1 (nb = min(nbw, s - k)) of [A | I] in
// one launch; block (i, q) writes row i of matrix q from buffer `par` into the
// other one.  Every block repeats, in LDS, the partial-pivoting elimination
// of the panel (columns k .. k + nb - 1 of the rows k .. s - 1).  Its pivots
// are the ones the step-by-step elimination chooses (largest modulus of the
// updated column, ties to the lower row; eliminating the rows above k does not
// change them), and its factors P_R = L_R U (P_R: the panel of the pivot rows
// in pivot order, L_R unit lower, U upper, nb x nb) give the rows after the nb
// steps directly: pivot row t becomes e_t U^-1 L_R^-1 times the old pivot
// rows, and any other row x its old row minus P_x U^-1 L_R^-1 times them
// (P_x: its panel).  Only the columns past the panel are written: the panel's
// own columns have become unit columns and are not read again.
constexpr int kGJPanel = 8;

__global__ __launch_bounds__(256) void gj_panel(GJBatch b, int k, int par, int nbw) {
  const GJMat M = b.m[blockIdx.y];
  const int s = M.s;
  const int i = blockIdx.x;  // this block's row
  if (k >= s || i >= s) return;
  const int nb = min(nbw, s - k);
  const int w = 2 * s;
  const int m = s - k;  // candidate rows k .. s - 1, local index r = row - k
  const cplx* A = M.a[par];
  cplx* O = M.a[par ^ 1];
  extern __shared__ double gj_lds[];
  cplx* V = reinterpret_cast<cplx*>(gj_lds);                // m x nbw panel, row-major
  int* orig = reinterpret_cast<int*>(V + (size_t)m * nbw);  // old row at each local position
  __shared__ cplx g[kGJPanel];  // coefficients of the old pivot rows in this block's row
  __shared__ int R[kGJPanel];   // old pivot rows, in pivot order
  __shared__ double bv[4];
  __shared__ int bi[4];
  const int tid = threadIdx.x;
  for (int r = tid; r < m; r += 256) {  // one row per thread: no division
    const cplx* ar = A + (size_t)(k + r) * w + k;
    for (int t = 0; t < nb; ++t) V[r * nbw + t] = ar[t];
    orig[r] = k + r;
  }
  __syncthreads();
  for (int t = 0; t < nb; ++t) {
    // pivot: wave-level argmax (ties to the lower row), then across the 4 waves
    double best = -1.0;
    int bidx = m;
    for (int r = t + tid; r < m; r += 256) {
      const cplx a = V[r * nbw + t];
      const double q = a.re * a.re + a.im * a.im;
      if (q > best) {
        best = q;
        bidx = r;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off);
      const int oi = __shfl_xor(bidx, off);
      if (o > best || (o == best && oi < bidx)) {
        best = o;
        bidx = oi;
      }
    }
    if ((tid & 63) == 0) {
      bv[tid >> 6] = best;
      bi[tid >> 6] = bidx;
    }
    __syncthreads();
    best = bv[0];
    int p = bi[0];
#pragma unroll
    for (int q = 1; q < 4; ++q)
      if (bv[q] > best || (bv[q] == best && bi[q] < p)) {
        best = bv[q];
        p = bi[q];
      }
    if (!(best > 0.0)) {  // the same in every thread and block of this matrix
      if (i == 0 && tid == 0) b.status[blockIdx.y] = 1;
      return;
    }
    if (p != t) {
      if (tid < nb) {
        const cplx x = V[p * nbw + tid];
        V[p * nbw + tid] = V[t * nbw + tid];
        V[t * nbw + tid] = x;
      }
      if (tid == 0) {
        const int x = orig[p];
        orig[p] = orig[t];
        orig[t] = x;
      }
    }
    __syncthreads();
    // eliminate column t below the pivot in the panel's later columns; the
    // column itself keeps the unnormalised multipliers (L = V / U_tt)
    const int nc = nb - t - 1;
    if (nc > 0) {
      const cplx pv = V[t * nbw + t];
      const double den = pv.re * pv.re + pv.im * pv.im;
      const cplx inv = {pv.re / den, -pv.im / den};
      for (int r = t + 1 + tid; r < m; r += 256) {  // one row per thread
        const cplx l = cmul(V[r * nbw + t], inv);
        for (int u = t + 1; u < nb; ++u) {
          const cplx pu = V[t * nbw + u];
          cplx& x = V[r * nbw + u];
          x = {x.re - (l.re * pu.re - l.im * pu.im), x.im - (l.re * pu.im + l.im * pu.re)};
        }
      }
    }
    __syncthreads();
  }
  // in parallel: 1/U_uu, L_R (below the diagonal) and the right-hand side
  // (e_t for pivot row t, else the panel of the old source row)
  __shared__ cplx Lr[kGJPanel * kGJPanel], invd[kGJPanel], rhs[kGJPanel];
  const bool piv = i >= k && i < k + nb;
  const int src = piv ? 0 : (i < k ? i : orig[i - k]);
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, u = e - r * nb;
    const cplx d = V[u * nbw + u];
    const double den = d.re * d.re + d.im * d.im;
    const cplx inv = {d.re / den, -d.im / den};
    if (r > u) Lr[e] = cmul(V[r * nbw + u], inv);
    if (r == u) invd[u] = inv;
  }
  if (tid < nb) rhs[tid] = piv ? cplx{tid == i - k ? 1.0 : 0.0, 0.0} : A[(size_t)src * w + k + tid];
  __syncthreads();
  if (tid == 0) {
    // y U = rhs, then c L_R = y; the row is alpha (old source row) + g (old pivot rows)
    cplx y[kGJPanel], c[kGJPanel];
    for (int u = 0; u < nb; ++u) {
      cplx acc = rhs[u];
      for (int v = 0; v < u; ++v) {
        const cplx uv = V[v * nbw + u];
        acc = {acc.re - (y[v].re * uv.re - y[v].im * uv.im), acc.im - (y[v].re * uv.im + y[v].im * uv.re)};
      }
      y[u] = cmul(acc, invd[u]);
    }
    for (int u = nb - 1; u >= 0; --u) {
      cplx acc = y[u];
      for (int r = u + 1; r < nb; ++r) {
        const cplx l = Lr[r * nb + u];
        acc = {acc.re - (c[r].re * l.re - c[r].im * l.im), acc.im - (c[r].re * l.im + c[r].im * l.re)};
      }
      c[u] = acc;
    }
    for (int u = 0; u < nb; ++u) {
      g[u] = piv ? c[u] : cplx{-c[u].re, -c[u].im};
      R[u] = orig[u];
    }
  }
  __syncthreads();
  const double alpha = piv ? 0.0 : 1.0;
  const cplx* srow = A + (size_t)src * w;
  cplx* orow = O + (size_t)i * w;
  cplx gg[kGJPanel];
  const cplx* prow[kGJPanel];
#pragma unroll
  for (int u = 0; u < kGJPanel; ++u) {
    gg[u] = u < nb ? g[u] : cplx{0.0, 0.0};
    prow[u] = A + (size_t)(u < nb ? R[u] : R[0]) * w;
  }
  for (int c = k + nb + tid; c < w; c += 256) {
    const cplx x = srow[c];
    cplx v = {alpha * x.re, alpha * x.im};
#pragma unroll
    for (int u = 0; u < kGJPanel; ++u) {
      if (u < nb) {
        const cplx pr = prow[u][c];
        v = {v.re + (gg[u].re * pr.re - gg[u].im * pr.im), v.im + (gg[u].re * pr.im + gg[u].im * pr.re)};
      }
    }
    orow[c] = v;
  }
}

// col[i] = A[i][0] of a row-major matrix with w columns
__global__ void copy_column(const cplx* __restrict__ A, cplx* col, int rows, int w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) col[i] = A[(size_t)i * w];
}

// [S | I] from a row-major K x K matrix S
__global__ void augment_identity(const cplx* __restrict__ S, cplx* A, int K) {
  const size_t tot = (size_t)K * 2 * K;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = idx / (2 * K), c = idx % (2 * K);
    A[idx] = c < K ? S[(size_t)r * K + c] : cplx{(c - K == r) ? 1.0 : 0.0, 0.0};
  }
}

// Inverts any number of matrices, eight per batch.
static int gj_batch(hipStream_t st, GJBatch& b, int count, DevBuf& status, int cap);
// cap: at most this many steps per launch (0: as many as fit, up to kGJPanel)
static int gj_invert(hipStream_t st, std::vector<GJMat>& mats, DevBuf& status, int cap) {
  for (size_t q0 = 0; q0 < mats.size(); q0 += 8) {
    GJBatch b{};
    const int count = (int)std::min<size_t>(8, mats.size() - q0);
    for (int q = 0; q < count; ++q) b.m[q] = mats[q0 + q];
    DP_TRY(gj_batch(st, b, count, status, cap));
    for (int q = 0; q < count; ++q) mats[q0 + q].res = b.m[q].res;
  }
  return DP_OK;
}

// Inverts the batch (at most 8 matrices): one launch per step of the largest.
static int gj_batch(hipStream_t st, GJBatch& b, int count, DevBuf& status, int cap) {
  DP_TRY(status.reserve(8 * sizeof(int)));
  b.status = status.as<int>();
  DP_HIP(hipMemsetAsync(b.status, 0, 8 * sizeof(int), st));
  int smax = 0;
  for (int q = 0; q < count; ++q) smax = std::max(smax, b.m[q].s);
  // panel width: the panel and the row map of the largest matrix in 63 KB of
  // LDS (with the kernel's own small arrays, under 64 KB)
  int nbw = cap > 0 ? std::min(cap, kGJPanel) : kGJPanel;
  while (nbw > 1 && (size_t)smax * (16 * nbw + 4) > 63 * 1024) nbw /= 2;
  if (nbw >= 2) {
    const size_t lds = (size_t)smax * (16 * nbw + 4);
    int launches = 0;
    for (int k = 0; k < smax; k += nbw, ++launches)
      gj_panel<<<dim3(smax, count), 256, lds, st>>>(b, k, launches & 1, nbw);
    for (int q = 0; q < count; ++q) b.m[q].res = ((b.m[q].s + nbw - 1) / nbw) & 1;
  } else {  // one launch per step
    for (int q = 0; q < count; ++q)  // pivot column of step 0
      copy_column<<<(b.m[q].s + 255) / 256, 256, 0, st>>>(b.m[q].a[0], b.m[q].col[0], b.m[q].s, 2 * b.m[q].s);
    for (int k = 0; k < smax; ++k) gj_step<<<dim3(smax, count), 256, 0, st>>>(b, k);
    for (int q = 0; q < count; ++q) b.m[q].res = b.m[q].s & 1;
  }
  DP_HIP(hipGetLastError());
  int h[8] = {0};
  DP_HIP(hipMemcpyAsync(h, b.status, 8 * sizeof(int), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  for (int q = 0; q < count; ++q)
    if (h[q]) {
      set_error("singular dense block in the preconditioner setup (size %d)", b.m[q].s);
      return DP_ESINGULAR;
    }
  return DP_OK;
}

// inverse of a row-major s x s matrix (given in the left half of Aug)
// ------------------------------------------------------------------ dense products
// C (M x N) = A (M x Kd) * B (Kd x N), all row-major (setup products).
__global__ void dense_gemm(const cplx* __restrict__ A, const cplx* __restrict__ B, cplx* C, int M, int N, int Kd) {
  const size_t tot = (size_t)M * N;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = idx / N, c = idx % N;
    cplx acc = {0.0, 0.0};
    for (int k = 0; k < Kd; ++k) cfma(acc, A[(size_t)r * Kd + k], B[(size_t)k * N + c]);
    C[idx] = acc;
  }
}

// U (s x K) and U^t (K x s): U(a, j) = exp(2 pi i (j - J)(a - (s-1)/2)/s)
__global__ void partial_fourier(cplx* U, cplx* Ut, int s, int J) {
  const int K = 2 * J + 1;
  const size_t tot = (size_t)s * K;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int a = idx / K, jj = idx % K;
    const int j = jj - J;
    // phase/pi = 2 j (a - (s-1)/2)/s = j (2a - s + 1)/s, reduced exactly mod 2
    long long num = (long long)j * (2LL * a - s + 1);
    long long den = s;
    long long r = num % (2 * den);
    double sn, cs;
    sincospi((double)r / (double)den, &sn, &cs);
    U[idx] = {cs, sn};
    Ut[(size_t)jj * s + a] = {cs, sn};
  }
}

// alpha_s(b) = (1/s) sum_a l_b(xi_a), xi_a = (a - (s-1)/2)/(s/2), Lagrange basis
// on first-kind Chebyshev points x_b = cos((2b+1) pi/(2 m_c)).
// One block per basis function b (256 threads over the s points).
__global__ __launch_bounds__(256) void lagrange_mean(double* alpha, int s, int mc) {
  __shared__ double xs[64];
  __shared__ double red[256];
  const int b = blockIdx.x;
  if (threadIdx.x < mc) xs[threadIdx.x] = cospi((2.0 * threadIdx.x + 1.0) / (2.0 * mc));
  __syncthreads();
  const double xb = xs[b];
  double acc = 0.0;
  for (int a = threadIdx.x; a < s; a += 256) {
    const double xa = (a - 0.5 * (s - 1)) / (0.5 * s);
    double num = 1.0, den = 1.0;
    for (int c = 0; c < mc; ++c) {
      if (c == b) continue;
      num *= xa - xs[c];
      den *= xb - xs[c];
    }
    acc += num / den;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) alpha[b] = red[0] / s;
}

// ------------------------------------------------------------------ geometry
// Trigonometric interpolant of the node positions at fractional node index u:
// x(u) = sum_j x_j D(u - j), D = (1/n) sin(pi (u-j)) cot(pi (u-j)/n) (modes
// |k| < n/2 plus the Nyquist cosine), and its derivative in the parameter.
// out[p] = {x, y, dx, dy} (derivative w.r.t. node index, direction only used).
__global__ __launch_bounds__(256) void trig_interp(const SrcRec* __restrict__ src, const double* __restrict__ u,
                                                   double* out, int n) {
  __shared__ double red[4][256];
  const double up = u[blockIdx.x];
  double ax = 0, ay = 0, dx = 0, dy = 0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double w = up - j;
    double sw, cw, sh, ch;
    sincospi(w, &sw, &cw);
    sincospi(w / n, &sh, &ch);
    double D, Dp;
    if (fabs(sh) < 1e-14) {
      D = 1.0;
      Dp = 0.0;
    } else {
      // D = sin(pi w) cot(pi w/n)/n ; dD/dw = [pi cos(pi w) cot(pi w/n) - (pi/n) sin(pi w)/sin^2(pi w/n)]/n
      D = sw * ch / sh / n;
      Dp = (kPi * cw * ch / sh - (kPi / n) * sw / (sh * sh)) / n;
    }
    const SrcRec s = src[j];
    ax = fma(s.x, D, ax);
    ay = fma(s.y, D, ay);
    dx = fma(s.x, Dp, dx);
    dy = fma(s.y, Dp, dy);
  }
  red[0][threadIdx.x] = ax;
  red[1][threadIdx.x] = ay;
  red[2][threadIdx.x] = dx;
  red[3][threadIdx.x] = dy;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

struct EArgs {
  const double* geo;     // per segment: (1 + m_c) points x {x, y, dx, dy}
  const int* seg;        // per segment: off, len, J, cls
  const double* alpha;   // per class m_c values (concatenated)
  cplx* e;               // per ordered pair (i, j != i), row-major in i
  int* kk;               // 2 per pair: k^i, k^j
  int m, mc, n;
  double omega, eta, ds;
  int kind;
};

// CFIE kernel without the identity part at (x, nx) <- (y, ny).
__device__ __forceinline__ cplx cfie_kernel(int kind, double omega, double eta, double x0, double x1, double nx0,
                                            double nx1, double y0, double y1, double ny0, double ny1) {
  const double d0 = x0 - y0, d1 = x1 - y1;
  const double r = sqrt(d0 * d0 + d1 * d1);
  const double r0 = d0 / r, r1 = d1 / r;
  const H01 h = hankel01(omega * r);
  if (kind == DP_SOFT) {
    // (i omega/4) H1 ny.rhat + (eta/4) H0
    const double a = 0.25 * omega * (ny0 * r0 + ny1 * r1);
    return {-a * h.h1.im + 0.25 * eta * h.h0.re, a * h.h1.re + 0.25 * eta * h.h0.im};
  }
  const double nxr = nx0 * r0 + nx1 * r1, nyr = ny0 * r0 + ny1 * r1, nn = nx0 * ny0 + nx1 * ny1;
  // hyp = (i omega/4) [ (omega H0 - 2 H1/r) nxr nyr + H1 nn / r ]
  const cplx inner = {(omega * h.h0.re - 2.0 * h.h1.re / r) * nxr * nyr + h.h1.re * nn / r,
                      (omega * h.h0.im - 2.0 * h.h1.im / r) * nxr * nyr + h.h1.im * nn / r};
  const cplx hyp = {-0.25 * omega * inner.im, 0.25 * omega * inner.re};
  // (i omega/4) H1 nxr + hyp/(i eta)
  const cplx a = {-0.25 * omega * nxr * h.h1.im, 0.25 * omega * nxr * h.h1.re};
  return {a.re + hyp.im / eta, a.im - hyp.re / eta};
}

// One block per ordered pair (i, j), i != j: directions and e_ij (eq. (14)).
__global__ __launch_bounds__(128) void e_entries(EArgs a) {
  __shared__ cplx red[128];
  __shared__ int kij[2];
  const int pair = blockIdx.x;
  const int i = pair / (a.m - 1);
  int j = pair % (a.m - 1);
  if (j >= i) ++j;
  const int mc = a.mc;
  const double* gi = a.geo + (size_t)i * (1 + mc) * 4;
  const double* gj = a.geo + (size_t)j * (1 + mc) * 4;
  const int si = a.seg[4 * i + 1], Ji = a.seg[4 * i + 2], ci = a.seg[4 * i + 3];
  const int sj = a.seg[4 * j + 1], Jj = a.seg[4 * j + 2], cj = a.seg[4 * j + 3];
  const double hi = 2.0 * kPi / (si * a.ds), hj = 2.0 * kPi / (sj * a.ds);
  if (threadIdx.x == 0) {
    double a0 = gi[0] - gj[0], a1 = gi[1] - gj[1];
    const double an = sqrt(a0 * a0 + a1 * a1);
    a0 /= an;
    a1 /= an;
    const double ti_n = sqrt(gi[2] * gi[2] + gi[3] * gi[3]);
    const double tj_n = sqrt(gj[2] * gj[2] + gj[3] * gj[3]);
    const double ati = (a0 * gi[2] + a1 * gi[3]) / ti_n;
    const double atj = (a0 * gj[2] + a1 * gj[3]) / tj_n;
    double ki = round_half_away(a.omega * ati / hi);
    double kj = round_half_away(-a.omega * atj / hj);
    ki = fmin(fmax(ki, -Ji), Ji);
    kj = fmin(fmax(kj, -Jj), Jj);
    kij[0] = (int)ki;
    kij[1] = (int)kj;
  }
  __syncthreads();
  const int ki = kij[0], kj = kij[1];
  const double* ali = a.alpha + (size_t)ci * mc;
  const double* alj = a.alpha + (size_t)cj * mc;
  cplx acc = {0.0, 0.0};
  for (int t = threadIdx.x; t < mc * mc; t += 128) {
    const int b = t / mc, bp = t % mc;
    const double* X = gi + 4 * (1 + b);
    const double* Y = gj + 4 * (1 + bp);
    const double tx = sqrt(X[2] * X[2] + X[3] * X[3]), ty = sqrt(Y[2] * Y[2] + Y[3] * Y[3]);
    // outward normal = (t_y, -t_x) for counter-clockwise nodes
    cplx M = cfie_kernel(a.kind, a.omega, a.eta, X[0], X[1], X[3] / tx, -X[2] / tx, Y[0], Y[1], Y[3] / ty,
                         -Y[2] / ty);
    M.re *= a.ds;
    M.im *= a.ds;
    // chebyshev offsets from the centres (arclength): delta = xi * s ds/2
    const double di = cospi((2.0 * b + 1.0) / (2.0 * mc)) * (0.5 * si * a.ds);
    const double dj = cospi((2.0 * bp + 1.0) / (2.0 * mc)) * (0.5 * sj * a.ds);
    double sn, cs;
    dp_sincos(-(ki * hi * di + kj * hj * dj), sn, cs);
    const cplx Mt = cmul(M, cplx{cs, sn});
    const double wgt = ali[b] * alj[bp];
    acc.re = fma(wgt, Mt.re, acc.re);
    acc.im = fma(wgt, Mt.im, acc.im);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 64; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[threadIdx.x].re += red[threadIdx.x + st].re;
      red[threadIdx.x].im += red[threadIdx.x + st].im;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.e[pair] = red[0];
    a.kk[2 * pair] = ki;
    a.kk[2 * pair + 1] = kj;
  }
}

// ------------------------------------------------------------------ apply kernels
template <class C>
struct SegGemm {
  const int* segs;     // per segment: off, len, offK, cls
  const C* const* A;   // per class: matrix pointer (row-major), chosen by `which`
  const int* dims;     // per class: s, K
  const C* X;          // input, column-major, leading dim ldx
  const C* Z;          // mode 1: out = Z - A X (leading dim ldy)
  C* Y;
  int ldx, ldy, nrhs;
  int mrows;           // 0: rows = s, 1: rows = K
  int kin;             // 0: inner dim = s (X rows at off), 1: inner = K (X rows at offK)
  int yoff;            // 0: Y rows at off, 1: at offK
  int mode;            // 0: Y = A X, 1: Y = Z - A X
};

// acc += a b for complex a, b of either precision
template <class C>
__device__ __forceinline__ void cfma_t(C& acc, C a, C b) {
  acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}

// Batched per-segment complex GEMM: grid (segment, row tile of 64, column
// tile of 16); the A tile and the X tile of each 16-deep slice go through LDS.
// C = cplx (FP64) or cplxf (the single-precision apply).
template <class C>
__global__ __launch_bounds__(256) void seg_gemm(SegGemm<C> g) {
  __shared__ C As[64][17];
  __shared__ C Xs[16][16];
  const int sg = blockIdx.x;
  const int off = g.segs[4 * sg], offK = g.segs[4 * sg + 2], cls = g.segs[4 * sg + 3];
  const int s = g.dims[2 * cls], K = g.dims[2 * cls + 1];
  const int M = g.mrows ? K : s;
  const int Kd = g.kin ? K : s;
  const int r0 = blockIdx.y * 64;
  if (r0 >= M) return;
  const int c0 = blockIdx.z * 16;
  const C* A = g.A[cls];
  const int xo = g.kin ? offK : off;
  const int yo = g.yoff ? offK : off;
  const int tr = threadIdx.x / 16;   // 0..15 -> rows tr, tr+16, tr+32, tr+48
  const int tc = threadIdx.x % 16;
  C acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int k0 = 0; k0 < Kd; k0 += 16) {
    for (int t = threadIdx.x; t < 64 * 16; t += 256) {
      const int rr = t / 16, kk = t % 16;
      const int r = r0 + rr, k = k0 + kk;
      As[rr][kk] = (r < M && k < Kd) ? A[(size_t)r * Kd + k] : C{0, 0};
    }
    {
      const int kk = threadIdx.x / 16, cc = threadIdx.x % 16;
      const int k = k0 + kk, c = c0 + cc;
      Xs[kk][cc] = (k < Kd && c < g.nrhs) ? g.X[(size_t)c * g.ldx + xo + k] : C{0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const C xv = Xs[kk][tc];
#pragma unroll
      for (int q = 0; q < 4; ++q) cfma_t(acc[q], As[tr + 16 * q][kk], xv);
    }
    __syncthreads();
  }
  const int c = c0 + tc;
  if (c >= g.nrhs) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + tr + 16 * q;
    if (r >= M) continue;
    const size_t o = (size_t)c * g.ldy + yo + r;
    if (g.mode == 1) {
      const C z = g.Z[o];
      g.Y[o] = {z.re - acc[q].re, z.im - acc[q].im};
    } else {
      g.Y[o] = acc[q];
    }
  }
}

// FP32 batched per-segment complex GEMM on the matrix cores
// (v_mfma_f32_16x16x4f32, A[i][k] in lane i + 16k, B[k][c] in lane c + 16k,
// D[i][c] in register r of lane c + 16 (i / 4), i = 4 (lane / 16) + r).
// Grid (segment, row tile of 64, column tile of 64); 4 waves, each 16 rows x
// 64 columns; the 64 x 16 A tile and the 16 x 64 X tile of each 16-deep
// slice go through LDS.  Complex products take 4 real ones:
// Re += Ar Xr + (-Ai) Xi, Im += Ar Xi + Ai Xr.
typedef float flt4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void seg_gemm_mfma32(SegGemm<cplxf> g) {
  __shared__ cplxf As[64][17];
  __shared__ cplxf Xs[16][65];
  const int sg = blockIdx.x;
  const int off = g.segs[4 * sg], offK = g.segs[4 * sg + 2], cls = g.segs[4 * sg + 3];
  const int s = g.dims[2 * cls], K = g.dims[2 * cls + 1];
  const int M = g.mrows ? K : s;
  const int Kd = g.kin ? K : s;
  const int r0 = blockIdx.y * 64;
  if (r0 >= M) return;
  const int c0 = blockIdx.z * 64;
  const cplxf* A = g.A[cls];
  const int xo = g.kin ? offK : off;
  const int yo = g.yoff ? offK : off;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  flt4v re[4], im[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    re[cb] = flt4v{0, 0, 0, 0};
    im[cb] = flt4v{0, 0, 0, 0};
  }
  // each thread moves 4 A and 4 X elements per 16-deep slice; the next
  // slice is requested before the current one's products
  cplxf ra[4], rx[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = threadIdx.x + 256 * q;
      const int rr = t >> 4, kk = t & 15;
      const int r = r0 + rr, k = k0 + kk;
      ra[q] = (r < M && k < Kd) ? A[(size_t)r * Kd + k] : cplxf{0, 0};
      const int c = c0 + rr;  // X: kk fastest, column rr
      rx[q] = (k < Kd && c < g.nrhs) ? g.X[(size_t)c * g.ldx + xo + k] : cplxf{0, 0};
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < Kd; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = threadIdx.x + 256 * q;
      As[t >> 4][t & 15] = ra[q];
      Xs[t & 15][t >> 4] = rx[q];
    }
    __syncthreads();
    if (k0 + 16 < Kd) fetch(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const cplxf a = As[16 * w + li][ks + lk];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const cplxf x = Xs[ks + lk][16 * cb + li];
        re[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, x.re, re[cb], 0, 0, 0);
        im[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, x.im, im[cb], 0, 0, 0);
        re[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.im, x.im, re[cb], 0, 0, 0);
        im[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, x.re, im[cb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = c0 + 16 * cb + li;
    if (c >= g.nrhs) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + 16 * w + 4 * lk + r;
      if (row >= M) continue;
      const size_t o = (size_t)c * g.ldy + yo + row;
      if (g.mode == 1) {
        const cplxf z = g.Z[o];
        g.Y[o] = {z.re - re[cb][r], z.im - im[cb][r]};
      } else {
        g.Y[o] = {re[cb][r], im[cb][r]};
      }
    }
  }
}

// Single-precision batched per-segment complex GEMM on the BF16 matrix cores.
// Every FP32 operand x is cut, by truncating masks, into three BF16 pieces
// x = h + m + l exactly (8 significant bits each); a real product keeps the
// six piece products of level h = 0, m = 1, l = 2 up to 2 (dropped terms are
// 2^-24 relative, like FP32 rounding) with FP32 accumulation, on
// v_mfma_f32_16x16x32_bf16 (A[i][k] in lane i + 16 (k / 8), element k % 8;
// B[k][c] in lane c + 16 (k / 8); D[i][c] in register i % 4 of lane
// c + 16 (i / 4)).  Grid (segment, row tile of 64, column tile of 64);
// 4 waves, each 16 rows x 64 columns; per 32-deep slice the A and X tiles
// are split into LDS as [piece][re/im][row or column][32 k], the four 16-byte
// chunks of a row stored at chunk ^ ((row / 4) % 4) so that 16 lanes reading
// one chunk of 16 rows hit distinct banks.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3_bf16(float x, uint32_t& h, uint32_t& m, uint32_t& l) {
  const uint32_t xb = __builtin_bit_cast(uint32_t, x);
  const float hf = __builtin_bit_cast(float, xb & 0xffff0000u);
  const float r = x - hf;  // exact: at most 16 significant bits remain
  const uint32_t rb = __builtin_bit_cast(uint32_t, r);
  const float mf = __builtin_bit_cast(float, rb & 0xffff0000u);
  const float lf = r - mf;  // exact, and exactly a BF16 value
  h = xb >> 16;
  m = rb >> 16;
  l = __builtin_bit_cast(uint32_t, lf) >> 16;
}

__device__ __forceinline__ flt4v mma_bf16(const uint4& a, const uint4& b, flt4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a), __builtin_bit_cast(bf16x8v, b), c,
                                                 0, 0, 0);
}

__global__ __launch_bounds__(256, 3) void seg_gemm_bf16x3(SegGemm<cplxf> g) {
  // [piece 3][re, im][64 rows or columns][16 words of two k]
  __shared__ __align__(16) uint32_t As[3][2][64][16];
  __shared__ __align__(16) uint32_t Xs[3][2][64][16];
  const int sg = blockIdx.x;
  const int off = g.segs[4 * sg], offK = g.segs[4 * sg + 2], cls = g.segs[4 * sg + 3];
  const int s = g.dims[2 * cls], K = g.dims[2 * cls + 1];
  const int M = g.mrows ? K : s;
  const int Kd = g.kin ? K : s;
  const int r0 = blockIdx.y * 64;
  if (r0 >= M) return;
  const int c0 = blockIdx.z * 64;
  const cplxf* A = g.A[cls];
  const int xo = g.kin ? offK : off;
  const int yo = g.yoff ? offK : off;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  flt4v re[4], im[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    re[cb] = flt4v{0, 0, 0, 0};
    im[cb] = flt4v{0, 0, 0, 0};
  }
  // each thread moves two consecutive k of four rows of A and four columns
  // of X per slice (word kp = k / 2 of row rr); the next slice is requested
  // before the current one's products
  cplxf ra[4][2], rx[4][2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, kp = e & 15;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = k0 + 2 * kp + h;
        const int r = r0 + rr, c = c0 + rr;
        ra[q][h] = (r < M && k < Kd) ? A[(size_t)r * Kd + k] : cplxf{0, 0};
        rx[q][h] = (k < Kd && c < g.nrhs) ? g.X[(size_t)c * g.ldx + xo + k] : cplxf{0, 0};
      }
    }
  };
  auto put = [&](uint32_t (&T)[3][2][64][16], int rr, int kp, const cplxf (&v)[2]) {
    const int pos = (((kp >> 2) ^ ((rr >> 2) & 3)) << 2) | (kp & 3);
    uint32_t h0, m0, l0, h1, m1, l1;
    split3_bf16(v[0].re, h0, m0, l0);
    split3_bf16(v[1].re, h1, m1, l1);
    T[0][0][rr][pos] = h0 | (h1 << 16);
    T[1][0][rr][pos] = m0 | (m1 << 16);
    T[2][0][rr][pos] = l0 | (l1 << 16);
    split3_bf16(v[0].im, h0, m0, l0);
    split3_bf16(v[1].im, h1, m1, l1);
    T[0][1][rr][pos] = h0 | (h1 << 16);
    T[1][1][rr][pos] = m0 | (m1 << 16);
    T[2][1][rr][pos] = l0 | (l1 << 16);
  };
  auto frag = [&](const uint32_t (&T)[3][2][64][16], int pc, int part, int rr) {
    const int pos = (lk ^ ((rr >> 2) & 3)) << 2;
    return *reinterpret_cast<const uint4*>(&T[pc][part][rr][pos]);
  };
  fetch(0);
  for (int k0 = 0; k0 < Kd; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      put(As, e >> 4, e & 15, ra[q]);
      put(Xs, e >> 4, e & 15, rx[q]);
    }
    __syncthreads();
    if (k0 + 32 < Kd) fetch(k0 + 32);
    uint4 ar[3], ai[3], an[3];
#pragma unroll
    for (int pc = 0; pc < 3; ++pc) {
      ar[pc] = frag(As, pc, 0, 16 * w + li);
      ai[pc] = frag(As, pc, 1, 16 * w + li);
      an[pc] = uint4{ai[pc].x ^ 0x80008000u, ai[pc].y ^ 0x80008000u, ai[pc].z ^ 0x80008000u,
                     ai[pc].w ^ 0x80008000u};
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      uint4 xr[3], xi[3];
#pragma unroll
      for (int pc = 0; pc < 3; ++pc) {
        xr[pc] = frag(Xs, pc, 0, 16 * cb + li);
        xi[pc] = frag(Xs, pc, 1, 16 * cb + li);
      }
      // piece pairs (a, x) with level a + x <= 2
#pragma unroll
      for (int pa = 0; pa < 3; ++pa) {
#pragma unroll
        for (int px = 0; px + pa < 3; ++px) {
          re[cb] = mma_bf16(ar[pa], xr[px], re[cb]);
          im[cb] = mma_bf16(ar[pa], xi[px], im[cb]);
          re[cb] = mma_bf16(an[pa], xi[px], re[cb]);
          im[cb] = mma_bf16(ai[pa], xr[px], im[cb]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = c0 + 16 * cb + li;
    if (c >= g.nrhs) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + 16 * w + 4 * lk + r;
      if (row >= M) continue;
      const size_t o = (size_t)c * g.ldy + yo + row;
      if (g.mode == 1) {
        const cplxf z = g.Z[o];
        g.Y[o] = {z.re - re[cb][r], z.im - im[cb][r]};
      } else {
        g.Y[o] = {re[cb][r], im[cb][r]};
      }
    }
  }
}

// precision conversions of n-element complex arrays
__global__ void to_single(const cplx* __restrict__ a, cplxf* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = {(float)a[i].re, (float)a[i].im};
}
__global__ void to_double(const cplxf* __restrict__ a, cplx* b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = {(double)a[i].re, (double)a[i].im};
}

__global__ void gather_rows(const cplx* __restrict__ z, cplx* zp, const int* __restrict__ perm, int NW, int nrhs) {
  const size_t tot = (size_t)NW * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int k = idx % NW, c = idx / NW;
    zp[idx] = z[(size_t)c * NW + perm[k]];
  }
}

__global__ void scatter_rows(const cplx* __restrict__ up, cplx* u, const int* __restrict__ perm, int NW, int nrhs) {
  const size_t tot = (size_t)NW * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int b = idx % NW, c = idx / NW;
    u[(size_t)c * NW + perm[b]] = up[idx];
  }
}

// Level-scheduled sparse triangular solve in place on x (NW x nrhs,
// column-major).  One block handles a group of columns; rows of one level
// are independent and are processed together, levels in order.
// lower: x_i -= sum_j L_ij x_j (unit diagonal); upper: x_i = (x_i - sum U_ij x_j)/U_ii.
__global__ __launch_bounds__(1024) void level_solve(cplx* x, const int* __restrict__ P, const int* __restrict__ Jc,
                                                    const cplx* __restrict__ V, const cplx* __restrict__ diag,
                                                    const int* __restrict__ lptr, const int* __restrict__ lrows,
                                                    int nlev, int NW, int nrhs, int cpb) {
  const int c0 = blockIdx.x * cpb;
  const int nc = min(cpb, nrhs - c0);
  for (int l = 0; l < nlev; ++l) {
    const int b = lptr[l], e = lptr[l + 1];
    const int items = (e - b) * nc;
    for (int t = threadIdx.x; t < items; t += blockDim.x) {
      const int ri = lrows[b + t / nc];
      const int c = c0 + t % nc;
      cplx* xc = x + (size_t)c * NW;
      cplx acc = xc[ri];
      for (int q = P[ri]; q < P[ri + 1]; ++q) {
        const cplx a = V[q], xv = xc[Jc[q]];
        acc.re -= a.re * xv.re - a.im * xv.im;
        acc.im -= a.re * xv.im + a.im * xv.re;
      }
      if (diag) {
        const cplx d = diag[ri];
        const double den = d.re * d.re + d.im * d.im;
        acc = {(acc.re * d.re + acc.im * d.im) / den, (acc.im * d.re - acc.re * d.im) / den};
      }
      xc[ri] = acc;
    }
    __syncthreads();
  }
}

// Whole floor(W)^{-1} z for one column per wave, the column held in LDS:
// gather zp[k] = z[perm_in[k]], forward solve with L (unit diagonal),
// backward solve with U, scatter u[perm_out[b]] = u'[b].  Both solves are
// one stream of steps of 64 slot records (col, row, value): a lane group of
// 1, 4, 16 or 64 lanes (chosen per level, coded in the top bits of col) works
// through rows of a dependency level one after another, one entry per lane
// per step, and the step that ends a row (row >= 0) writes x[row] = sum of
// value * x[col] over the row's slots (lane sums by DPP moves only).  A row's slots
// hold its own diagonal term (x[row] times 1 or 1/U_rr) and the negated,
// scaled off-diagonal entries, so every row is a plain dot product; rows of
// one level are independent, and a level's steps come after all steps of the
// levels it depends on.  One wave executes its LDS accesses in program order,
// so no barrier is needed, and the slot loads run 32 steps ahead.
// Steps go in batches of kTriBatch that never span two levels (each level's
// steps are padded to a multiple of the batch with empty steps of its lane
// width): no step of a batch reads an element another step of it writes, so
// the batch's LDS reads are issued together, then its accumulations, its
// lane sums (independent chains, one width for the batch) and its writes.
// (Skipping the sums of batches in which no row ends cost more than it saved.)
constexpr int kSlotAhead = 32;  // steps the slot loads run ahead (one wave per CU: registers to spare)
constexpr int kTriBatch = 4;    // steps per batch (divides kSlotAhead)
static_assert(kSlotAhead % kTriBatch == 0, "batches must tile the prefetch round");

// Value of the lane given by a DPP control: quad permutations 0xB1 (l ^ 1)
// and 0x4E (l ^ 2), rotations within a row of 16 lanes 0x124 (by 4) and
// 0x128 (by 8), and the row broadcasts 0x142 (lane 15 of the row below, in
// the rows of ROWS) and 0x143 (lane 31, rows of ROWS); rows outside ROWS get 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_sum(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_sum(double v) {
  const int2 h = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, int2{__builtin_amdgcn_update_dpp(0, h.x, CTRL, ROWS, 0xF, false),
                                         __builtin_amdgcn_update_dpp(0, h.y, CTRL, ROWS, 0xF, false)});
}

template <class C>
struct Slot {
  int col, row;
  decltype(C{}.re) re, im;
};

template <class C>
__global__ __launch_bounds__(64) void tri_solve_wave(const C* __restrict__ z, C* __restrict__ u, int NW,
                                                     const int* __restrict__ pin, const int* __restrict__ pout,
                                                     const Slot<C>* __restrict__ slots, int nsteps) {
  extern __shared__ unsigned char lds_raw[];
  C* xs = reinterpret_cast<C*>(lds_raw);  // NW + 1 elements
  const size_t c = blockIdx.x;
  const int lane = threadIdx.x;
#pragma unroll 32
  for (int k = lane; k < NW; k += 64) xs[k] = z[c * NW + pin[k]];
  // nsteps is a multiple of D and the stream holds D more padding steps
  constexpr int D = kSlotAhead;
  Slot<C> ring[D];
#pragma unroll
  for (int q = 0; q < D; ++q) ring[q] = slots[(size_t)q * 64 + lane];
  C acc = {0, 0};
  // the lane holding a row's total: the lane itself for one lane per row,
  // the first of its group of 4 or 16 lanes, or lane 48 (row 3) for a
  // 64-lane row
  const bool head4 = (lane & 3) == 0, head16 = (lane & 15) == 0, head64 = lane == 48;
  for (int s0 = 0; s0 < nsteps; s0 += D) {
#pragma unroll
    for (int q0 = 0; q0 < D; q0 += kTriBatch) {
      constexpr int B = kTriBatch;
      Slot<C> r[B];
      C xv[B], tot[B];
#pragma unroll
      for (int b = 0; b < B; ++b) r[b] = ring[q0 + b];
#pragma unroll
      for (int b = 0; b < B; ++b) xv[b] = xs[r[b].col & 0x3fffffff];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        acc.re = fma(r[b].re, xv[b].re, fma(-r[b].im, xv[b].im, acc.re));
        acc.im = fma(r[b].re, xv[b].im, fma(r[b].im, xv[b].re, acc.im));
        tot[b] = acc;
        const bool fin = r[b].row >= 0;
        acc.re = fin ? 0 : acc.re;
        acc.im = fin ? 0 : acc.im;
      }
      // lane sums and writes only for a batch in which some row ends (the
      // steps of a long row before its last one just accumulate)
      // the batch's lanes per row (1, 4, 16 or 64) are in bits 30..31 of col
      const int wcode = __builtin_amdgcn_readfirstlane((int)((unsigned)r[0].col >> 30));
      if (wcode) {  // 4 lanes: quad permutations
#pragma unroll
        for (int b = 0; b < B; ++b) {
          tot[b].re += dpp_sum<0xB1>(tot[b].re);  // lanes 4g + (l ^ 1)
          tot[b].im += dpp_sum<0xB1>(tot[b].im);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
          tot[b].re += dpp_sum<0x4E>(tot[b].re);  // lanes 4g + (l ^ 2)
          tot[b].im += dpp_sum<0x4E>(tot[b].im);
        }
        if (wcode > 1) {  // 16 lanes: rotations by 4 and 8 within the row
#pragma unroll
          for (int b = 0; b < B; ++b) {
            tot[b].re += dpp_sum<0x124>(tot[b].re);
            tot[b].im += dpp_sum<0x124>(tot[b].im);
          }
#pragma unroll
          for (int b = 0; b < B; ++b) {
            tot[b].re += dpp_sum<0x128>(tot[b].re);
            tot[b].im += dpp_sum<0x128>(tot[b].im);
          }
          if (wcode > 2) {  // 64 lanes: rows 1, 3 += rows 0, 2; then rows 2, 3 += row 1
#pragma unroll
            for (int b = 0; b < B; ++b) {
              tot[b].re += dpp_sum<0x142, 0xA>(tot[b].re);
              tot[b].im += dpp_sum<0x142, 0xA>(tot[b].im);
            }
#pragma unroll
            for (int b = 0; b < B; ++b) {
              tot[b].re += dpp_sum<0x143, 0xC>(tot[b].re);
              tot[b].im += dpp_sum<0x143, 0xC>(tot[b].im);
            }
          }
        }
      }
      const bool head = wcode == 0 ? true : (wcode == 1 ? head4 : (wcode == 2 ? head16 : head64));
      // branch-free: lanes that do not finish a row write the spare element xs[NW]
#pragma unroll
      for (int b = 0; b < B; ++b) xs[r[b].row >= 0 && head ? r[b].row : NW] = tot[b];
      // the ring entries are reloaded after their last use, so that each
      // load can write the registers it replaces (no copies, and no wait for
      // the newest loads, at the end of a round)
#pragma unroll
      for (int b = 0; b < B; ++b) ring[q0 + b] = slots[(size_t)(s0 + q0 + b + D) * 64 + lane];
    }
  }
#pragma unroll 32
  for (int k = lane; k < NW; k += 64) u[c * NW + pout[k]] = xs[k];
}

// Step stream of the forward (L) then backward (U) solve: within each level,
// rows sorted by slot count are dealt longest first to the least-loaded lane
// group, with 1, 4, 16 or 64 lanes per row, whichever takes the fewest steps
// (long rows alone in a level use the whole wave); each level's steps are
// padded to whole batches of kTriBatch.  Padding slots have column 0 (with the
// level's width code), value 0 and row -1.
template <class C>
static int build_slots(const SparseLU& lu, std::vector<Slot<C>>& out) {
  using R = decltype(C{}.re);
  const int NW = lu.n;
  out.clear();
  out.reserve((size_t)(lu.Lx.size() + lu.Ux.size() + 2 * NW) / 8 * 64);
  std::vector<std::pair<int, std::complex<double>>> ent;
  int steps = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<int>& lptr = pass ? lu.lvlU_ptr : lu.lvlL_ptr;
    const std::vector<int>& lrows = pass ? lu.lvlU_rows : lu.lvlL_rows;
    const std::vector<int>& Pp = pass ? lu.Up : lu.Lp;
    const std::vector<int>& Jj = pass ? lu.Uj : lu.Lj;
    const auto& Vv = pass ? lu.Ux : lu.Lx;
    const int nlev = (int)lptr.size() - 1;
    for (int l = 0; l < nlev; ++l) {
      std::vector<std::pair<int, int>> rows;  // (slot count, row)
      for (int q = lptr[l]; q < lptr[l + 1]; ++q) {
        const int r = lrows[q];
        rows.push_back({Pp[r + 1] - Pp[r] + 1, r});
      }
      std::sort(rows.begin(), rows.end(), [](const auto& a, const auto& b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
      });
      // lanes per row W in {1, 4, 16, 64}: the one with the fewest steps
      // once they are padded to whole batches
      int best_w = 1, best_st = INT32_MAX;
      std::vector<std::vector<int>> best_grp;
      for (int W : {1, 4, 16, 64}) {
        const int ng = 64 / W;
        std::vector<std::vector<int>> grp(ng);
        // least-loaded group first, ties to the lower group index
        std::priority_queue<std::pair<int, int>, std::vector<std::pair<int, int>>, std::greater<>> heap;
        for (int g = 0; g < ng; ++g) heap.push({0, g});
        int maxload = 0;
        for (const auto& [cnt, r] : rows) {
          auto [ld, g] = heap.top();
          heap.pop();
          grp[g].push_back(r);
          ld += (cnt + W - 1) / W;
          maxload = std::max(maxload, ld);
          heap.push({ld, g});
        }
        const int nst = (maxload + kTriBatch - 1) / kTriBatch * kTriBatch;
        if (nst < best_st) {
          best_st = nst;
          best_w = W;
          best_grp = std::move(grp);
        }
      }
      const int W = best_w, nst = best_st;
      const int wcode = W == 1 ? 0 : (W == 4 ? 1 : (W == 16 ? 2 : 3));
      const size_t base = out.size();
      out.resize(base + (size_t)nst * 64, Slot<C>{wcode << 30, -1, 0, 0});
      for (int g = 0; g < 64 / W; ++g) {
        int st = 0;
        for (int r : best_grp[g]) {
          const std::complex<double> d = pass ? 1.0 / lu.Ud[r] : std::complex<double>(1.0, 0.0);
          ent.clear();
          ent.push_back({r, d});
          for (int q = Pp[r]; q < Pp[r + 1]; ++q) ent.push_back({Jj[q], -d * Vv[q]});
          const int rs = ((int)ent.size() + W - 1) / W;
          for (int k = 0; k < rs; ++k)
            for (int lr = 0; lr < W; ++lr) {
              Slot<C>& sl = out[base + (size_t)(st + k) * 64 + W * g + lr];
              const int e = W * k + lr;
              if (e < (int)ent.size()) {
                sl.col = ent[e].first | (wcode << 30);
                sl.re = (R)ent[e].second.real();
                sl.im = (R)ent[e].second.imag();
              }
              sl.row = (k == rs - 1) ? r : -1;
            }
          st += rs;
        }
      }
      steps += nst;
    }
  }
  // round up to whole prefetch rounds, plus one round that is only loaded
  const int total = (steps + kSlotAhead - 1) / kSlotAhead * kSlotAhead;
  out.resize((size_t)(total + kSlotAhead) * 64, Slot<C>{0, -1, 0, 0});  // width code 0
  (void)NW;
  return total;
}

// ------------------------------------------------------------------ host: setup
static void segment_boundary(const dp_problem* p, const dp_precond_opts* o, std::vector<int>& off,
                             std::vector<int>& len) {
  const int n = (int)p->n;
  const double L = p->L, ds = L / n, lam = 2.0 * kPi / p->omega;
  int m0 = 1 << (int)std::lround(std::log2(std::sqrt(L / lam)));
  m0 = std::max(1, std::min(m0, n));
  while (n % m0) m0 /= 2;
  std::vector<std::pair<int, int>> st;
  const int s0 = n / m0;
  for (int t = m0 - 1; t >= 0; --t) st.push_back({t * s0, s0});
  while (!st.empty()) {
    auto [o0, s] = st.back();
    st.pop_back();
    double cmax = 0;
    for (int a = o0; a < o0 + s; ++a) cmax = std::max(cmax, std::fabs(p->hkap[a]));
    const double length = s * ds;
    if (cmax == 0 || length <= std::sqrt(L * lam / cmax) || length <= o->m_ell * lam || s <= o->min_pts || s % 2) {
      off.push_back(o0);
      len.push_back(s);
      continue;
    }
    st.push_back({o0 + s / 2, s / 2});
    st.push_back({o0, s / 2});
  }
}

static void threshold_T(const std::vector<cplx>& T, int K, double t_keep, std::vector<cplx>& Tt) {
  Tt = T;
  if (t_keep <= 0) return;
  const int k = (int)std::min<long long>((long long)K * K, std::llround(t_keep * K));
  std::vector<double> mag(T.size());
  for (size_t q = 0; q < T.size(); ++q) mag[q] = std::hypot(T[q].re, T[q].im);
  std::vector<double> srt(mag);
  std::nth_element(srt.begin(), srt.begin() + (k - 1), srt.end(), std::greater<double>());
  const double tau = srt[k - 1];
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) {
      const size_t q = (size_t)r * K + c;
      const bool keep = mag[q] >= tau * (1 - 1e-8) || c == K - 1 - r;
      if (!keep) Tt[q] = {0.0, 0.0};
    }
}

int precond_build(dp_problem* p, const dp_precond_opts* o) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = p->ctx->stream;
  // A rebuild takes over the previous preconditioner's device buffers:
  // those already large enough are reused rather than freed and allocated
  // again (each hipFree waits for the device).  Its graphs and host state
  // are not kept.
  Precond* old = p->pc;
  p->pc = nullptr;
  Precond* P = new Precond();
  auto take = [](DevBuf& dst, DevBuf& src) {
    dst = src;
    src = DevBuf{};
  };
  if (old) {
    for (auto pr : {std::make_pair(&P->d_segs, &old->d_segs), std::make_pair(&P->d_ptrs, &old->d_ptrs),
                    std::make_pair(&P->d_ptrs32, &old->d_ptrs32), std::make_pair(&P->d_dims, &old->d_dims),
                    std::make_pair(&P->Lp, &old->Lp), std::make_pair(&P->Lj, &old->Lj),
                    std::make_pair(&P->Lx, &old->Lx), std::make_pair(&P->Up, &old->Up),
                    std::make_pair(&P->Uj, &old->Uj), std::make_pair(&P->Ux, &old->Ux),
                    std::make_pair(&P->Ud, &old->Ud), std::make_pair(&P->lvlL, &old->lvlL),
                    std::make_pair(&P->lvlLr, &old->lvlLr), std::make_pair(&P->lvlU, &old->lvlU),
                    std::make_pair(&P->lvlUr, &old->lvlUr), std::make_pair(&P->pin, &old->pin),
                    std::make_pair(&P->pout, &old->pout), std::make_pair(&P->slots, &old->slots),
                    std::make_pair(&P->slots32, &old->slots32), std::make_pair(&P->wy, &old->wy),
                    std::make_pair(&P->wg, &old->wg), std::make_pair(&P->wz, &old->wz),
                    std::make_pair(&P->wu, &old->wu), std::make_pair(&P->wt, &old->wt),
                    std::make_pair(&P->wn, &old->wn), std::make_pair(&P->sy, &old->sy),
                    std::make_pair(&P->sg, &old->sg), std::make_pair(&P->sz, &old->sz),
                    std::make_pair(&P->su, &old->su), std::make_pair(&P->sn, &old->sn),
                    std::make_pair(&P->sv, &old->sv), std::make_pair(&P->sq, &old->sq),
                    std::make_pair(&P->win, &old->win), std::make_pair(&P->wq, &old->wq)})
      take(*pr.first, *pr.second);
  }
  auto drop_old = [&]() {
    if (old) precond_destroy(old);
    old = nullptr;
  };
  auto fail = [&](int rc) {
    drop_old();
    precond_destroy(P);
    return rc;
  };
  const int n = (int)p->n;
  const double L = p->L, ds = L / n, omega = p->omega;
  P->m_c = o->m_c;
  P->graphs = o->graphs != 0;
  segment_boundary(p, o, P->off, P->len);
  P->m = (int)P->off.size();
  const int m = P->m;
  if (m < 2) {
    set_error("dp_precond_build: fewer than two segments");
    return fail(DP_EINVAL);
  }
  std::map<int, int> cls_of;
  for (int s : P->len) cls_of[s] = 0;
  for (auto& kv : cls_of) {
    kv.second = (int)P->classes.size();
    SizeClass c;
    c.s = kv.first;
    c.J = (int)std::ceil(c.s * omega * ds / (2.0 * kPi) - 1e-9);
    c.K = 2 * c.J + 1;
    P->classes.push_back(std::move(c));
  }
  if (old) {  // per-class buffers, by class index
    for (size_t ci = 0; ci < std::min(P->classes.size(), old->classes.size()); ++ci) {
      SizeClass& c = P->classes[ci];
      SizeClass& oc = old->classes[ci];
      for (auto pr : {std::make_pair(&c.Binv, &oc.Binv), std::make_pair(&c.U, &oc.U), std::make_pair(&c.Ut, &oc.Ut),
                      std::make_pair(&c.Tt, &oc.Tt), std::make_pair(&c.alpha, &oc.alpha),
                      std::make_pair(&c.Binv32, &oc.Binv32), std::make_pair(&c.U32, &oc.U32),
                      std::make_pair(&c.Ut32, &oc.Ut32), std::make_pair(&c.Tt32, &oc.Tt32)})
        take(*pr.first, *pr.second);
    }
  }
  drop_old();
  P->offK.assign(m + 1, 0);
  P->cls.resize(m);
  P->J.resize(m);
  for (int i = 0; i < m; ++i) {
    P->cls[i] = cls_of[P->len[i]];
    P->J[i] = P->classes[P->cls[i]].J;
    P->offK[i + 1] = P->offK[i] + P->classes[P->cls[i]].K;
  }
  P->NW = P->offK[m];
  const int mc = o->m_c;

  // ---- size classes: B^{-1}, U, S, T, floor(T), alpha (batched over classes)
  const int ncls = (int)P->classes.size();
  // per class (so that no class's buffer is reallocated while a kernel of
  // the previous class may still read it, and the loops need no waits)
  std::vector<DevBuf> augB(2 * ncls), augS(2 * ncls), colB(2 * ncls), colS(2 * ncls), rows(ncls), Xs(ncls),
      Ss(ncls);
  DevBuf gstat;
  DevBuf d_alpha;
  struct Release {  // the setup's own buffers, on every return path
    std::vector<DevBuf*> bufs;
    std::vector<DevBuf>* vecs[7];
    ~Release() {
      for (DevBuf* q : bufs) q->release();
      for (auto* v : vecs)
        for (DevBuf& q : *v) q.release();
    }
  } release_locals{{&gstat, &d_alpha}, {&augB, &augS, &colB, &colS, &rows, &Xs, &Ss}};
  DP_TRY(d_alpha.reserve(ncls * mc * sizeof(double)));
  std::vector<GJMat> gb(ncls);
  for (int ci = 0; ci < ncls; ++ci)
    lagrange_mean<<<mc, 256, 0, st>>>(d_alpha.as<double>() + ci * mc, P->classes[ci].s, mc);
  // ---- segment geometry: centre + m_c Chebyshev points, by trigonometric interpolation
  const int npts = m * (1 + mc);
  std::vector<double> uh(npts);
  for (int i = 0; i < m; ++i) {
    const double uc = P->off[i] + 0.5 * (P->len[i] - 1);
    uh[(size_t)i * (1 + mc)] = uc;
    for (int b = 0; b < mc; ++b) {
      const double xi = std::cos((2.0 * b + 1.0) * kPi / (2.0 * mc));
      double u = uc + xi * 0.5 * P->len[i];
      if (u < 0) u += n;
      if (u >= n) u -= n;
      uh[(size_t)i * (1 + mc) + 1 + b] = u;
    }
  }
  DevBuf d_u, d_geo, d_seg, d_e, d_kk;
  std::vector<int> seg4(4 * m);
  for (int i = 0; i < m; ++i) {
    seg4[4 * i] = P->off[i];
    seg4[4 * i + 1] = P->len[i];
    seg4[4 * i + 2] = P->J[i];
    seg4[4 * i + 3] = P->cls[i];
  }
  const size_t npair = (size_t)m * (m - 1);
  int rc;
  if ((rc = upload(d_u, uh, st)) || (rc = d_geo.reserve((size_t)npts * 4 * sizeof(double))) ||
      (rc = upload(d_seg, seg4, st)) || (rc = d_e.reserve(npair * sizeof(cplx))) ||
      (rc = d_kk.reserve(npair * 2 * sizeof(int))))
    return fail(rc);
  trig_interp<<<npts, 256, 0, st>>>(p->src.as<SrcRec>(), d_u.as<double>(), d_geo.as<double>(), n);
  EArgs ea;
  ea.geo = d_geo.as<double>();
  ea.seg = d_seg.as<int>();
  ea.alpha = d_alpha.as<double>();
  ea.e = d_e.as<cplx>();
  ea.kk = d_kk.as<int>();
  ea.m = m;
  ea.mc = mc;
  ea.n = n;
  ea.omega = omega;
  ea.eta = p->eta;
  ea.ds = ds;
  ea.kind = p->kind;
  e_entries<<<(unsigned)npair, 128, 0, st>>>(ea);
  DP_HIP(hipGetLastError());
  P->eval.resize(npair);
  std::vector<int> kk(npair * 2);
  DP_HIP(hipMemcpyAsync(P->eval.data(), d_e.p, npair * sizeof(cplx), hipMemcpyDeviceToHost, st));
  DP_HIP(hipMemcpyAsync(kk.data(), d_kk.p, npair * 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  P->eidx.resize(npair * 4);
  for (size_t q = 0; q < npair; ++q) {
    const int i = (int)(q / (m - 1));
    int j = (int)(q % (m - 1));
    if (j >= i) ++j;
    P->eidx[4 * q] = i;
    P->eidx[4 * q + 1] = j;
    P->eidx[4 * q + 2] = kk[2 * q];
    P->eidx[4 * q + 3] = kk[2 * q + 1];
  }

  // ---- pattern of floor(W) = E + antidiag(T) in CSC; each stored entry
  // keeps the list of its sources (an antidiagonal entry of T_i, coded
  // -(offK_i + r) - 1, or the E entry q), summed in that order once T is known
  const int NW = P->NW;
  std::vector<int> cp(NW + 1, 0), ri, ssrc_ptr(1, 0), ssrc;
  {
    std::vector<std::vector<std::pair<int, int>>> cols(NW);  // (row, source)
    for (int i = 0; i < m; ++i) {
      const int K = P->classes[P->cls[i]].K;
      for (int r = 0; r < K; ++r) cols[P->offK[i] + K - 1 - r].push_back({P->offK[i] + r, -(P->offK[i] + r) - 1});
    }
    for (size_t q = 0; q < npair; ++q) {
      const int i = P->eidx[4 * q], j = P->eidx[4 * q + 1];
      const int row_ = P->offK[i] + P->eidx[4 * q + 2] + P->J[i];
      const int col_ = P->offK[j] + P->eidx[4 * q + 3] + P->J[j];
      cols[col_].push_back({row_, (int)q});
    }
    for (int c = 0; c < NW; ++c) {
      auto& v = cols[c];
      std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      for (size_t q = 0; q < v.size(); ++q) {
        // an E entry landing on an antidiagonal position is added to it
        if (q == 0 || v[q].first != v[q - 1].first) {
          ri.push_back(v[q].first);
          ssrc_ptr.push_back(ssrc_ptr.back());
        }
        ssrc.push_back(v[q].second);
        ssrc_ptr.back()++;
      }
      cp[c + 1] = (int)ri.size();
    }
  }
  P->nnzW = (int64_t)ri.size();
  // Host sparse LU unless the ordering predicts more than 32 factor entries
  // per row (many segments coupled all-to-all through E): then the sparse
  // solves are slower than dense ones and the host factorisation takes
  // seconds, so floor(W) is factored densely on the device instead.
  // With more than 2 N_W pair entries (m (m - 1) > 2 N_W) the coupling is
  // all-to-all enough that the ordering need not be tried.  The ordering
  // needs only the pattern: it runs on a host thread while the device
  // inverts the size classes.
  const int64_t fill_cap = o->w_solver == 1 ? INT64_MAX : 32 * (int64_t)NW;
  const bool go_dense = o->w_solver == 2 || (o->w_solver == 0 && (int64_t)m * (m - 1) > 2 * (int64_t)NW);
  std::vector<int> order;
  struct Joiner {
    std::thread t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } ordering;
  if (!go_dense) {
    try {
      ordering.t = std::thread([&] { order = sparse_lu_order(NW, cp, ri, fill_cap); });
    } catch (const std::system_error&) {  // no thread available: order now
      order = sparse_lu_order(NW, cp, ri, fill_cap);
    }
  }

  for (int ci = 0; ci < ncls; ++ci) {
    SizeClass& c = P->classes[ci];
    const int s = c.s, K = c.K;
    int rc;
    DevBuf& row = rows[ci];
    if ((rc = row.reserve(s * sizeof(cplx))) || (rc = augB[2 * ci].reserve((size_t)s * 2 * s * sizeof(cplx))) ||
        (rc = augB[2 * ci + 1].reserve((size_t)s * 2 * s * sizeof(cplx))) ||
        (rc = colB[2 * ci].reserve((size_t)s * sizeof(cplx))) || (rc = colB[2 * ci + 1].reserve((size_t)s * sizeof(cplx))) ||
        (rc = c.Binv.reserve((size_t)s * s * sizeof(cplx))) || (rc = c.U.reserve((size_t)s * K * sizeof(cplx))) ||
        (rc = c.Ut.reserve((size_t)s * K * sizeof(cplx))) || (rc = c.Tt.reserve((size_t)K * K * sizeof(cplx))))
      return fail(rc);
    flat_row<<<(s + 255) / 256, 256, 0, st>>>(p->C.as<double>(), row.as<cplx>(), s, n, L, omega, p->eta, p->kind);
    toeplitz_aug<<<grid1((size_t)s * 2 * s), 256, 0, st>>>(row.as<cplx>(), augB[2 * ci].as<cplx>(), s);
    gb[ci] = GJMat{{augB[2 * ci].as<cplx>(), augB[2 * ci + 1].as<cplx>()},
                   {colB[2 * ci].as<cplx>(), colB[2 * ci + 1].as<cplx>()}, s, 0};
  }
  {
    int rc;
    if ((rc = gj_invert(st, gb, gstat, o->gj_steps))) return fail(rc);
  }
  std::vector<GJMat> gs(ncls);
  for (int ci = 0; ci < ncls; ++ci) {
    SizeClass& c = P->classes[ci];
    const int s = c.s, K = c.K;
    copy_right_half<<<grid1((size_t)s * s), 256, 0, st>>>(augB[2 * ci + gb[ci].res].as<cplx>(), c.Binv.as<cplx>(), s);
    DevBuf &X = Xs[ci], &S = Ss[ci];
    int rc;
    if ((rc = X.reserve((size_t)s * K * sizeof(cplx))) || (rc = S.reserve((size_t)K * K * sizeof(cplx))) ||
        (rc = augS[2 * ci].reserve((size_t)K * 2 * K * sizeof(cplx))) ||
        (rc = augS[2 * ci + 1].reserve((size_t)K * 2 * K * sizeof(cplx))) ||
        (rc = colS[2 * ci].reserve((size_t)K * sizeof(cplx))) || (rc = colS[2 * ci + 1].reserve((size_t)K * sizeof(cplx))))
      return fail(rc);
    partial_fourier<<<grid1((size_t)s * K), 256, 0, st>>>(c.U.as<cplx>(), c.Ut.as<cplx>(), s, c.J);
    dense_gemm<<<grid1((size_t)s * K), 256, 0, st>>>(c.Binv.as<cplx>(), c.U.as<cplx>(), X.as<cplx>(), s, K, s);
    // S = U^t X, then [S | I]
    dense_gemm<<<grid1((size_t)K * K), 256, 0, st>>>(c.Ut.as<cplx>(), X.as<cplx>(), S.as<cplx>(), K, K, s);
    augment_identity<<<grid1((size_t)K * 2 * K), 256, 0, st>>>(S.as<cplx>(), augS[2 * ci].as<cplx>(), K);
    gs[ci] = GJMat{{augS[2 * ci].as<cplx>(), augS[2 * ci + 1].as<cplx>()},
                   {colS[2 * ci].as<cplx>(), colS[2 * ci + 1].as<cplx>()}, K, 0};
  }
  {
    int rc;
    if ((rc = gj_invert(st, gs, gstat, o->gj_steps))) return fail(rc);
  }
  // T_s to the host for all classes, one wait, threshold, back for all
  for (int ci = 0; ci < ncls; ++ci) {
    SizeClass& c = P->classes[ci];
    const int K = c.K;
    copy_right_half<<<grid1((size_t)K * K), 256, 0, st>>>(augS[2 * ci + gs[ci].res].as<cplx>(), c.Tt.as<cplx>(), K);
    c.T.resize((size_t)K * K);
    DP_HIP(hipMemcpyAsync(c.T.data(), c.Tt.p, c.T.size() * sizeof(cplx), hipMemcpyDeviceToHost, st));
  }
  DP_HIP(hipStreamSynchronize(st));
  {
    std::vector<std::vector<cplx>> Tts(ncls);
    for (int ci = 0; ci < ncls; ++ci) {
      SizeClass& c = P->classes[ci];
      threshold_T(c.T, c.K, o->t_keep, Tts[ci]);
      DP_HIP(hipMemcpyAsync(c.Tt.p, Tts[ci].data(), Tts[ci].size() * sizeof(cplx), hipMemcpyHostToDevice, st));
    }
    DP_HIP(hipStreamSynchronize(st));
  }
  DP_HIP(hipGetLastError());

  // ---- values of floor(W) (sources summed in their stored order); LU
  std::vector<zc> vx(ri.size());
  for (size_t e = 0; e < ri.size(); ++e) {
    zc v = 0.0;
    for (int q = ssrc_ptr[e]; q < ssrc_ptr[e + 1]; ++q) {
      const int src = ssrc[q];
      if (src < 0) {
        const int a = -src - 1;  // offK_i + r
        const int i = (int)(std::upper_bound(P->offK.begin(), P->offK.end(), a) - P->offK.begin()) - 1;
        const SizeClass& c = P->classes[P->cls[i]];
        const int r = a - P->offK[i];
        const cplx t = c.T[(size_t)r * c.K + (c.K - 1 - r)];
        v += zc(t.re, t.im);
      } else {
        v += zc(P->eval[src].re, P->eval[src].im);
      }
    }
    vx[e] = v;
  }
  if (ordering.t.joinable()) ordering.t.join();
  if (go_dense || (order.empty() && NW > 0)) rc = kSparseFillLimit;
  else rc = sparse_lu_factor_ordered(NW, cp, ri, vx, order, P->lu, fill_cap);
  if (rc == kSparseFillLimit) {
    if ((double)NW * NW * sizeof(cplx) > 48.0 * (1 << 30)) {
      set_error("floor(W) of dimension %d needs a dense factorisation larger than 48 GiB", NW);
      return fail(DP_ENOMEM);
    }
    std::vector<int> rows_, cols_;
    std::vector<cplx> vals_;
    rows_.reserve(ri.size());
    cols_.reserve(ri.size());
    vals_.reserve(ri.size());
    for (int c = 0; c < NW; ++c)
      for (int q = cp[c]; q < cp[c + 1]; ++q) {
        rows_.push_back(ri[q]);
        cols_.push_back(c);
        vals_.push_back({vx[q].real(), vx[q].imag()});
      }
    if ((rc = P->dlu.assemble(st, NW, rows_, cols_, vals_)) || (rc = P->dlu.factor(st))) return fail(rc);
    P->dense_w = true;
  } else if (rc) {
    return fail(rc);
  } else {
    auto to_c = [](const std::vector<zc>& a) {
      std::vector<cplx> r(a.size());
      for (size_t q = 0; q < a.size(); ++q) r[q] = {a[q].real(), a[q].imag()};
      return r;
    };
    const SparseLU& lu = P->lu;
    if ((rc = upload(P->Lp, lu.Lp, st)) || (rc = upload(P->Lj, lu.Lj, st)) || (rc = upload(P->Lx, to_c(lu.Lx), st)) ||
        (rc = upload(P->Up, lu.Up, st)) || (rc = upload(P->Uj, lu.Uj, st)) || (rc = upload(P->Ux, to_c(lu.Ux), st)) ||
        (rc = upload(P->Ud, to_c(lu.Ud), st)) || (rc = upload(P->lvlL, lu.lvlL_ptr, st)) ||
        (rc = upload(P->lvlLr, lu.lvlL_rows, st)) || (rc = upload(P->lvlU, lu.lvlU_ptr, st)) ||
        (rc = upload(P->lvlUr, lu.lvlU_rows, st)) || (rc = upload(P->pin, lu.perm_in, st)) ||
        (rc = upload(P->pout, lu.perm_out, st)))
      return fail(rc);
    P->nlevL = (int)lu.lvlL_ptr.size() - 1;
    P->nlevU = (int)lu.lvlU_ptr.size() - 1;
    {
      std::vector<Slot<cplx>> sl;
      P->nsteps = build_slots(lu, sl);
      std::vector<Slot<cplxf>> sl32(sl.size());
      for (size_t q = 0; q < sl.size(); ++q) sl32[q] = {sl[q].col, sl[q].row, (float)sl[q].re, (float)sl[q].im};
      if ((rc = upload(P->slots, sl, st)) || (rc = upload(P->slots32, sl32, st))) return fail(rc);
      int maxlds = 0;
      DP_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->ctx->device));
      P->lds_solve = (size_t)(NW + 1) * sizeof(cplx) <= (size_t)maxlds;
      P->lds_solve32 = (size_t)(NW + 1) * sizeof(cplxf) <= (size_t)maxlds;
      if (P->lds_solve)
        DP_HIP(hipFuncSetAttribute((const void*)tri_solve_wave<cplx>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)((NW + 1) * sizeof(cplx))));
      if (P->lds_solve32)
        DP_HIP(hipFuncSetAttribute((const void*)tri_solve_wave<cplxf>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)((NW + 1) * sizeof(cplxf))));
    }
  }

  // ---- apply tables
  std::vector<int> segs(4 * m), dims(2 * P->classes.size());
  std::vector<const cplx*> ptrs(4 * P->classes.size());
  for (int i = 0; i < m; ++i) {
    segs[4 * i] = P->off[i];
    segs[4 * i + 1] = P->len[i];
    segs[4 * i + 2] = P->offK[i];
    segs[4 * i + 3] = P->cls[i];
  }
  const size_t nc = P->classes.size();
  for (size_t c = 0; c < nc; ++c) {
    dims[2 * c] = P->classes[c].s;
    dims[2 * c + 1] = P->classes[c].K;
    ptrs[0 * nc + c] = P->classes[c].Binv.as<cplx>();
    ptrs[1 * nc + c] = P->classes[c].U.as<cplx>();
    ptrs[2 * nc + c] = P->classes[c].Ut.as<cplx>();
    ptrs[3 * nc + c] = P->classes[c].Tt.as<cplx>();
  }
  if ((rc = upload(P->d_segs, segs, st)) || (rc = upload(P->d_dims, dims, st)) ||
      (rc = upload(P->d_ptrs, ptrs, st)))
    return fail(rc);
  {
    std::vector<const cplxf*> ptrs32(4 * nc);
    for (size_t c = 0; c < nc; ++c) {
      SizeClass& sc = P->classes[c];
      const size_t ns = (size_t)sc.s * sc.s, nk = (size_t)sc.s * sc.K, kk = (size_t)sc.K * sc.K;
      if ((rc = sc.Binv32.reserve(ns * sizeof(cplxf))) || (rc = sc.U32.reserve(nk * sizeof(cplxf))) ||
          (rc = sc.Ut32.reserve(nk * sizeof(cplxf))) || (rc = sc.Tt32.reserve(kk * sizeof(cplxf))))
        return fail(rc);
      to_single<<<grid1(ns), 256, 0, st>>>(sc.Binv.as<cplx>(), sc.Binv32.as<cplxf>(), ns);
      to_single<<<grid1(nk), 256, 0, st>>>(sc.U.as<cplx>(), sc.U32.as<cplxf>(), nk);
      to_single<<<grid1(nk), 256, 0, st>>>(sc.Ut.as<cplx>(), sc.Ut32.as<cplxf>(), nk);
      to_single<<<grid1(kk), 256, 0, st>>>(sc.Tt.as<cplx>(), sc.Tt32.as<cplxf>(), kk);
      ptrs32[0 * nc + c] = sc.Binv32.as<cplxf>();
      ptrs32[1 * nc + c] = sc.U32.as<cplxf>();
      ptrs32[2 * nc + c] = sc.Ut32.as<cplxf>();
      ptrs32[3 * nc + c] = sc.Tt32.as<cplxf>();
    }
    if ((rc = upload(P->d_ptrs32, ptrs32, st))) return fail(rc);
  }
  DP_HIP(hipStreamSynchronize(st));
  gstat.release();
  d_alpha.release();
  d_u.release();
  d_geo.release();
  d_seg.release();
  d_e.release();
  d_kk.release();
  P->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  p->pc = P;
  return DP_OK;
}

// ------------------------------------------------------------------ host: apply
template <class C>
static int run_seg_gemm(dp_problem* p, int which, int mrows, int kin, int yoff, int mode, const C* X, int ldx,
                        const C* Z, C* Y, int ldy, int nrhs) {
  Precond* P = p->pc;
  const size_t nc = P->classes.size();
  int maxM = 0;
  for (auto& c : P->classes) maxM = std::max(maxM, mrows ? c.K : c.s);
  SegGemm<C> g;
  g.segs = P->d_segs.as<int>();
  g.A = (sizeof(C) == sizeof(cplx) ? P->d_ptrs.as<const C*>() : P->d_ptrs32.as<const C*>()) + which * nc;
  g.dims = P->d_dims.as<int>();
  g.X = X;
  g.Z = Z;
  g.Y = Y;
  g.ldx = ldx;
  g.ldy = ldy;
  g.nrhs = nrhs;
  g.mrows = mrows;
  g.kin = kin;
  g.yoff = yoff;
  g.mode = mode;
  if constexpr (sizeof(C) == sizeof(cplxf)) {
    if (nrhs >= 16) {
      dim3 grid(P->m, (maxM + 63) / 64, (nrhs + 63) / 64);
      seg_gemm_bf16x3<<<grid, 256, 0, p->ctx->stream>>>(g);
      DP_HIP(hipGetLastError());
      return DP_OK;
    }
  }
  dim3 grid(P->m, (maxM + 63) / 64, (nrhs + 15) / 16);
  seg_gemm<C><<<grid, 256, 0, p->ctx->stream>>>(g);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// u = floor(W)^{-1} z in FP64 (dense device LU, LDS-resident sparse solve, or
// the level-scheduled sparse solve)
// with the workspaces t (level-scheduled solve) and dt, dy (dense solve),
// each NW x nrhs; kernel launches only
static int w_solve_ws(dp_problem* p, int nrhs, const cplx* z, cplx* u, cplx* t, cplx* dt, cplx* dy) {
  Precond* P = p->pc;
  hipStream_t st = p->ctx->stream;
  const int NW = P->NW;
  if (P->dense_w) return P->dlu.solve_ws(st, z, u, nrhs, dt, dy);
  if (P->lds_solve) {
    tri_solve_wave<cplx><<<nrhs, 64, (size_t)(NW + 1) * sizeof(cplx), st>>>(
        z, u, NW, P->pin.as<int>(), P->pout.as<int>(), P->slots.as<Slot<cplx>>(), P->nsteps);
    return DP_OK;
  }
  gather_rows<<<grid1((size_t)NW * nrhs), 256, 0, st>>>(z, t, P->pin.as<int>(), NW, nrhs);
  const int cpb = nrhs < 16 ? nrhs : 16;
  const int nb = (nrhs + cpb - 1) / cpb;
  level_solve<<<nb, 1024, 0, st>>>(t, P->Lp.as<int>(), P->Lj.as<int>(), P->Lx.as<cplx>(), nullptr,
                                   P->lvlL.as<int>(), P->lvlLr.as<int>(), P->nlevL, NW, nrhs, cpb);
  level_solve<<<nb, 1024, 0, st>>>(t, P->Up.as<int>(), P->Uj.as<int>(), P->Ux.as<cplx>(), P->Ud.as<cplx>(),
                                   P->lvlU.as<int>(), P->lvlUr.as<int>(), P->nlevU, NW, nrhs, cpb);
  scatter_rows<<<grid1((size_t)NW * nrhs), 256, 0, st>>>(t, u, P->pout.as<int>(), NW, nrhs);
  return DP_OK;
}

// u = floor(W)^{-1} z with the preconditioner's own workspaces (the dense
// solve grows its workspaces as needed)
static int w_solve(dp_problem* p, int nrhs, const cplx* z, cplx* u) {
  Precond* P = p->pc;
  if (P->dense_w) return P->dlu.solve(p->ctx->stream, z, u, nrhs);
  return w_solve_ws(p, nrhs, z, u, P->wt.as<cplx>(), nullptr, nullptr);
}

// Workspaces of one FP64 apply for nrhs columns: y, un (n x nrhs); g, z, u,
// t, and for a dense floor(W) dt, dy (NW x nrhs)
struct ApplyWs {
  cplx *y, *un, *g, *z, *u, *t, *dt, *dy;
};

// eq. (19) on nrhs columns, kernels only (no allocation, no host sync): the
// sequence that is captured into a graph, and the apply of the entry point
// that allocates nothing.
static int apply_core_ws(dp_problem* p, int nrhs, const cplx* v, cplx* q, const ApplyWs& w) {
  Precond* P = p->pc;
  const int n = (int)p->n, NW = P->NW;
  cplx *y = w.y, *g = w.g, *z = w.z, *u = w.u, *un = w.un;
  enum { BINV = 0, UU = 1, UT = 2, TT = 3 };
  // y = B^{-1} v
  DP_TRY(run_seg_gemm<cplx>(p, BINV, 0, 0, 0, 0, v, n, nullptr, y, n, nrhs));
  // g = U^t y
  DP_TRY(run_seg_gemm<cplx>(p, UT, 1, 0, 1, 0, y, n, nullptr, g, NW, nrhs));
  // z = floor(T) g
  DP_TRY(run_seg_gemm<cplx>(p, TT, 1, 1, 1, 0, g, NW, nullptr, z, NW, nrhs));
  // u = floor(W)^{-1} z
  DP_TRY(w_solve_ws(p, nrhs, z, u, w.t, w.dt, w.dy));
  // h = z - floor(T) u  (into g)
  DP_TRY(run_seg_gemm<cplx>(p, TT, 1, 1, 1, 1, u, NW, z, g, NW, nrhs));
  // un = U h
  DP_TRY(run_seg_gemm<cplx>(p, UU, 0, 1, 0, 0, g, NW, nullptr, un, n, nrhs));
  // q = y - B^{-1} un
  DP_TRY(run_seg_gemm<cplx>(p, BINV, 0, 0, 0, 1, un, n, y, q, n, nrhs));
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// The FP64 apply on the preconditioner's workspaces (sized by precond_apply)
static int apply_core(dp_problem* p, int nrhs, const cplx* v, cplx* q) {
  Precond* P = p->pc;
  const ApplyWs w{P->wy.as<cplx>(), P->wn.as<cplx>(), P->wg.as<cplx>(), P->wz.as<cplx>(),
                  P->wu.as<cplx>(), P->wt.as<cplx>(), P->dlu.tws.as<cplx>(), P->dlu.yws.as<cplx>()};
  return apply_core_ws(p, nrhs, v, q, w);
}

// The same sequence with single-precision tables and vectors (FP64 in and
// out).  floor(W) is solved with its single-precision sparse factors in LDS
// when they fit, otherwise in FP64 between conversions.
static int apply_core32(dp_problem* p, int nrhs, const cplx* v, cplx* q) {
  Precond* P = p->pc;
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n, NW = P->NW;
  const size_t nn = (size_t)n * nrhs, nw = (size_t)NW * nrhs;
  cplxf *sv = P->sv.as<cplxf>(), *y = P->sy.as<cplxf>(), *g = P->sg.as<cplxf>(), *z = P->sz.as<cplxf>(),
        *u = P->su.as<cplxf>(), *un = P->sn.as<cplxf>(), *sq = P->sq.as<cplxf>();
  enum { BINV = 0, UU = 1, UT = 2, TT = 3 };
  to_single<<<grid1(nn), 256, 0, st>>>(v, sv, nn);
  DP_TRY(run_seg_gemm<cplxf>(p, BINV, 0, 0, 0, 0, sv, n, nullptr, y, n, nrhs));
  DP_TRY(run_seg_gemm<cplxf>(p, UT, 1, 0, 1, 0, y, n, nullptr, g, NW, nrhs));
  DP_TRY(run_seg_gemm<cplxf>(p, TT, 1, 1, 1, 0, g, NW, nullptr, z, NW, nrhs));
  if (!P->dense_w && P->lds_solve32) {
    tri_solve_wave<cplxf><<<nrhs, 64, (size_t)(NW + 1) * sizeof(cplxf), st>>>(
        z, u, NW, P->pin.as<int>(), P->pout.as<int>(), P->slots32.as<Slot<cplxf>>(), P->nsteps);
  } else {
    to_double<<<grid1(nw), 256, 0, st>>>(z, P->wz.as<cplx>(), nw);
    DP_TRY(w_solve(p, nrhs, P->wz.as<cplx>(), P->wu.as<cplx>()));
    to_single<<<grid1(nw), 256, 0, st>>>(P->wu.as<cplx>(), u, nw);
  }
  DP_TRY(run_seg_gemm<cplxf>(p, TT, 1, 1, 1, 1, u, NW, z, g, NW, nrhs));
  DP_TRY(run_seg_gemm<cplxf>(p, UU, 0, 1, 0, 0, g, NW, nullptr, un, n, nrhs));
  DP_TRY(run_seg_gemm<cplxf>(p, BINV, 0, 0, 0, 1, un, n, y, sq, n, nrhs));
  to_double<<<grid1(nn), 256, 0, st>>>(sq, q, nn);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// Capture one of the apply sequences on the workspace input/output into an
// executable graph.
static int capture_apply(dp_problem* p, int nrhs, int prec, hipGraphExec_t* out) {
  Precond* P = p->pc;
  hipStream_t st = p->ctx->stream;
  hipGraph_t g = nullptr;
  CaptureScope excl;  // no stream-ordered allocation in any thread until instantiated
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return DP_EDEVICE;
  const int rc = prec ? apply_core32(p, nrhs, P->win.as<cplx>(), P->wq.as<cplx>())
                      : apply_core(p, nrhs, P->win.as<cplx>(), P->wq.as<cplx>());
  const hipError_t e = hipStreamEndCapture(st, &g);
  hipGraphExec_t x = nullptr;
  const bool ok = rc == DP_OK && e == hipSuccess && g && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (!ok) return DP_EDEVICE;
  *out = x;
  return DP_OK;
}

// z = P v in FP64 (prec 0) or with the single-precision tables (prec 1, the
// correction solves of the mixed-precision solve).  The first call for a
// column count runs eagerly (and sizes the workspaces); the next one captures
// the kernel sequence into a HIP graph, which later calls replay between a
// copy of v into the graph's input buffer and a copy of its output into z:
// one launch instead of a dozen (sparse floor(W)) to a few hundred (dense
// floor(W)).  If capture fails that apply stays eager.
int precond_apply(dp_problem* p, int nrhs, const cplx* v, cplx* q, int prec) {
  Precond* P = p->pc;
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n, NW = P->NW;
  const size_t bn = (size_t)n * nrhs * sizeof(cplx), bw = (size_t)NW * nrhs * sizeof(cplx);
  DP_TRY(P->wy.reserve(bn));
  DP_TRY(P->wn.reserve(bn));
  DP_TRY(P->wg.reserve(bw));
  DP_TRY(P->wz.reserve(bw));
  DP_TRY(P->wu.reserve(bw));
  DP_TRY(P->wt.reserve(bw));
  if (P->dense_w) {
    DP_TRY(P->dlu.tws.reserve(bw));
    DP_TRY(P->dlu.yws.reserve(bw));
  }
  if (prec) {
    const size_t sn = bn / 2, sw = bw / 2;
    DP_TRY(P->sv.reserve(sn));
    DP_TRY(P->sy.reserve(sn));
    DP_TRY(P->sn.reserve(sn));
    DP_TRY(P->sq.reserve(sn));
    DP_TRY(P->sg.reserve(sw));
    DP_TRY(P->sz.reserve(sw));
    DP_TRY(P->su.reserve(sw));
  }
  bool& on = prec ? P->graphs32 : P->graphs;
  hipGraphExec_t& gx = prec ? P->gexec32 : P->gexec;
  int& gn = prec ? P->g32_nrhs : P->g_nrhs;
  int& gc = prec ? P->g32_calls : P->g_calls;
  std::vector<void*>& gsig = prec ? P->g32_sig : P->g_sig;
  auto eager = [&]() { return prec ? apply_core32(p, nrhs, v, q) : apply_core(p, nrhs, v, q); };
  if (!P->graphs || !on) return eager();
  // a graph holds the workspace addresses it was captured with: a different
  // column count or any workspace reallocated since (also by the other
  // precision's apply) means capturing again
  auto sig = [&]() {
    return std::vector<void*>{P->wy.p, P->wn.p, P->wg.p, P->wz.p, P->wu.p, P->wt.p, P->sv.p, P->sy.p,
                              P->sn.p, P->sq.p, P->sg.p, P->sz.p, P->su.p, P->win.p, P->wq.p,
                              P->dlu.tws.p, P->dlu.yws.p};
  };
  if (gn != nrhs || (gx && sig() != gsig)) {
    if (gx) (void)hipGraphExecDestroy(gx);
    gx = nullptr;
    gc = gn == nrhs ? 1 : 0;
    gn = nrhs;
  }
  if (!gx && gc++ >= 1) {
    // both precisions' graphs read and write win and wq (never in flight together)
    DP_TRY(P->win.reserve(bn));
    DP_TRY(P->wq.reserve(bn));
    if (capture_apply(p, nrhs, prec, &gx) != DP_OK) on = false;
    else gsig = sig();
  }
  if (!gx) return eager();
  DP_TRY(dev_copy(P->win.p, v, bn, st));
  DP_HIP(hipGraphLaunch(gx, st));
  DP_TRY(dev_copy(q, P->wq.p, bn, st));
  return DP_OK;
}

// ------------------------------------------------------------------ apply without allocation
// Device scratch of dp_precond_apply_noalloc: one array on every GPU the
// library runs on, resident until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: kernels receive the
// address that hipGetSymbolAddress returned for the device (scratch_base).
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_base;  // per device ordinal, nullptr until looked up

int scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_base.size() <= device) g_scratch_base.resize(device + 1, nullptr);
  if (g_scratch_base[device]) return DP_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    set_error("scratch address on device %d: %s", device, hipGetErrorString(e));
    return DP_EDEVICE;
  }
  g_scratch_base[device] = ptr;
  return DP_OK;
}

static void* scratch_base(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device < (int)g_scratch_base.size() ? g_scratch_base[device] : nullptr;
}

size_t scratch_bytes() { return kScratchBytes; }

// The FP64 apply of precond_apply with every workspace carved from the
// device's scratch array: kernel launches only, no allocation, no graph.
// Each workspace is written before it is read, so nothing is cleared.
int precond_apply_noalloc(dp_problem* p, int nrhs, const cplx* v, cplx* q) {
  Precond* P = p->pc;
  char* base = static_cast<char*>(scratch_base(p->ctx->device));
  if (!base) {
    set_error("dp_precond_apply_noalloc: no scratch address for device %d", p->ctx->device);
    return DP_EDEVICE;
  }
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t bn = al((size_t)p->n * nrhs * sizeof(cplx)), bw = al((size_t)P->NW * nrhs * sizeof(cplx));
  const size_t need = 2 * bn + (P->dense_w ? 6 : 4) * bw;
  if (need > kScratchBytes) {
    set_error("dp_precond_apply_noalloc: %d columns at n = %lld, NW = %d need %zu bytes of scratch; the maximum "
              "is %zu",
              nrhs, (long long)p->n, P->NW, need, kScratchBytes);
    return DP_EINVAL;
  }
  ApplyWs w{};
  char* c = base;
  for (cplx** slot : {&w.y, &w.un}) {
    *slot = reinterpret_cast<cplx*>(c);
    c += bn;
  }
  for (cplx** slot : {&w.g, &w.z, &w.u, &w.t}) {
    *slot = reinterpret_cast<cplx*>(c);
    c += bw;
  }
  if (P->dense_w) {
    w.dt = reinterpret_cast<cplx*>(c);
    w.dy = reinterpret_cast<cplx*>(c + bw);
  }
  return apply_core_ws(p, nrhs, v, q, w);
}

void precond_destroy(Precond* P) {
  if (!P) return;
  for (auto& c : P->classes) {
    c.Binv.release();
    c.U.release();
    c.Ut.release();
    c.Tt.release();
    c.alpha.release();
  }
  for (DevBuf* b : {&P->d_segs, &P->d_ptrs, &P->d_dims, &P->Lp, &P->Lj, &P->Lx, &P->Up, &P->Uj, &P->Ux, &P->Ud,
                    &P->lvlL, &P->lvlLr, &P->lvlU, &P->lvlUr, &P->pin, &P->pout, &P->wy, &P->wg, &P->wz, &P->wu,
                    &P->wt, &P->wn, &P->slots, &P->slots32})
    b->release();
  P->dlu.release();
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->gexec32) (void)hipGraphExecDestroy(P->gexec32);
  for (auto& c : P->classes) {
    c.Binv32.release();
    c.U32.release();
    c.Ut32.release();
    c.Tt32.release();
  }
  for (DevBuf* b : {&P->d_ptrs32, &P->sy, &P->sg, &P->sz, &P->su, &P->sn,
                    &P->sv, &P->sq})
    b->release();
  P->win.release();
  P->wq.release();
  delete P;
}

int precond_info(dp_problem* p, dp_precond_info* info) {
  const Precond* P = p->pc;
  info->m = P->m;
  info->n_classes = (int64_t)P->classes.size();
  info->NW = P->NW;
  info->nnzE = (int64_t)P->m * (P->m - 1);
  info->nnzW = P->nnzW;
  info->nnzLU = P->dense_w ? (int64_t)P->NW * P->NW : (int64_t)P->lu.Lx.size() + (int64_t)P->lu.Ux.size() + P->NW;
  info->levels = P->dense_w ? 0 : P->nlevL + P->nlevU;
  info->dense_w = P->dense_w ? 1 : 0;
  info->t_setup = P->t_setup;
  return DP_OK;
}

int precond_export(dp_problem* p, int64_t* seg_off, int64_t* seg_len, int64_t* e_idx, double* e_val) {
  const Precond* P = p->pc;
  for (int i = 0; i < P->m; ++i) {
    if (seg_off) seg_off[i] = P->off[i];
    if (seg_len) seg_len[i] = P->len[i];
  }
  const size_t npair = (size_t)P->m * (P->m - 1);
  for (size_t q = 0; q < npair; ++q) {
    if (e_idx)
      for (int t = 0; t < 4; ++t) e_idx[4 * q + t] = P->eidx[4 * q + t];
    if (e_val) {
      e_val[2 * q] = P->eval[q].re;
      e_val[2 * q + 1] = P->eval[q].im;
    }
  }
  return DP_OK;
}

}  // namespace dp
