// Restarted GMRES for A q = f with nrhs independent columns (Sec. 3: GMRES,
// restart 80, relative tolerance).  Right preconditioning is done in the
// flexible form: z_k = P v_k is stored and the iterate is x = x0 + Z y, so no
// extra preconditioner application is needed and the residual is the true
// one.  Arnoldi uses classical Gram-Schmidt applied twice (CGS2) so that each
// step is two block dot-product / update sweeps over the basis.
//
// The whole Arnoldi step runs on the device: after the orthogonalisation,
// one block per column applies the column's previous Givens rotations to the
// new Hessenberg column, forms the next rotation, updates the least-squares
// right-hand side g and its residual estimate |g_{k+1}| / ||f||, stops the
// column when the estimate meets tol (or on breakdown, or at max_iters), and
// sets the scale 1/h_{k+1,k} of the next basis vector (0 for a stopped
// column).  The step index lives in device memory, so one captured HIP graph
// of the orthogonalisation and rotation kernels serves every step of every
// cycle (two graphs: basis sizes up to 16 fuse the first update with the
// second projection).  The host never waits for a step before queuing the
// next one: it reads the column states of step k-1 back (a small
// asynchronous copy) while step k runs, and queues step k+1 unless step k-1
// left no column running.  A step queued after every column stopped
// (found one step late) costs its preconditioner apply and matrix-vector
// product launches, whose pair sweep returns at once (guard flags), and
// changes no state; when the residual estimates predict that step k may stop
// the last columns, the host waits for step k before queuing more.  At the
// end of a cycle y = R^{-1} g is solved per column on the device and
// x += Z y; at each restart the true residual f - A x is recomputed and
// decides convergence.
#include <chrono>
#include <thread>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dp_internal.hpp"

namespace dp {

constexpr int kDotRows = 2048;

// partial[(bx * ps + i) * nrhs + c] = sum_{rows of block bx} conj(V_i[c]) W[c]
// for i <= *kd (the step index in device memory)
__global__ __launch_bounds__(256) void gram_dots(const cplx* __restrict__ V, size_t vstride,
                                                 const cplx* __restrict__ W, int n, int nrhs, const int* kd, int ps,
                                                 cplx* __restrict__ partial) {
  // eight basis vectors per pass over the rows; each sum is reduced within
  // its wave by a fixed butterfly, then over the four waves in order
  constexpr int G = 8;
  __shared__ cplx red[4][G];
  const int kp1 = *kd + 1;
  const int c = blockIdx.y;
  const int j0 = blockIdx.x * kDotRows;
  const int j1 = min(n, j0 + kDotRows);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const cplx* w = W + (size_t)c * n;
  for (int i0 = 0; i0 < kp1; i0 += G) {
    const int g = min(G, kp1 - i0);
    cplx s[G];
#pragma unroll
    for (int u = 0; u < G; ++u) s[u] = {0.0, 0.0};
    for (int j = j0 + threadIdx.x; j < j1; j += 256) {
      const cplx b = w[j];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (u < g) {
          const cplx a = V[(i0 + u) * vstride + (size_t)c * n + j];
          s[u].re = fma(a.re, b.re, fma(a.im, b.im, s[u].re));
          s[u].im = fma(a.re, b.im, fma(-a.im, b.re, s[u].im));
        }
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        s[u].re += __shfl_xor(s[u].re, off);
        s[u].im += __shfl_xor(s[u].im, off);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < G; ++u) red[wv][u] = s[u];
    }
    __syncthreads();
    if ((int)threadIdx.x < g) {
      const int u = threadIdx.x;
      cplx t = red[0][u];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        t.re += red[q][u].re;
        t.im += red[q][u].im;
      }
      partial[((size_t)blockIdx.x * ps + i0 + u) * nrhs + c] = t;
    }
    __syncthreads();
  }
}

// The first projection's update and the second projection's dot products in
// one pass over the basis, for basis sizes *kd + 1 <= kFuseK: per row,
// W[c] -= sum_i V_i[c] h[i][c] with the row's basis values held in registers,
// then the partial sums conj(V_i[c]) W[c] of the updated row, reduced as in
// gram_dots.  The grid is that of gram_dots.
constexpr int kFuseK = 16;

__global__ __launch_bounds__(256) void gram_update_dots(const cplx* __restrict__ V, size_t vstride,
                                                        cplx* __restrict__ W, const cplx* __restrict__ h, int n,
                                                        int nrhs, const int* kd, int ps, cplx* __restrict__ partial) {
  __shared__ cplx red[4][kFuseK];
  const int kp1 = *kd + 1;
  const int c = blockIdx.y;
  const int j0 = blockIdx.x * kDotRows;
  const int j1 = min(n, j0 + kDotRows);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cplx* w = W + (size_t)c * n;
  cplx hc[kFuseK], s[kFuseK];
#pragma unroll
  for (int u = 0; u < kFuseK; ++u) {
    hc[u] = u < kp1 ? h[u * nrhs + c] : cplx{0.0, 0.0};
    s[u] = {0.0, 0.0};
  }
  for (int j = j0 + threadIdx.x; j < j1; j += 256) {
    cplx a[kFuseK];
    cplx acc = w[j];
#pragma unroll
    for (int u = 0; u < kFuseK; ++u) {
      if (u < kp1) {
        a[u] = V[u * vstride + (size_t)c * n + j];
        acc.re -= a[u].re * hc[u].re - a[u].im * hc[u].im;
        acc.im -= a[u].re * hc[u].im + a[u].im * hc[u].re;
      }
    }
    w[j] = acc;
#pragma unroll
    for (int u = 0; u < kFuseK; ++u) {
      if (u < kp1) {
        s[u].re = fma(a[u].re, acc.re, fma(a[u].im, acc.im, s[u].re));
        s[u].im = fma(a[u].re, acc.im, fma(-a[u].im, acc.re, s[u].im));
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kFuseK; ++u) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s[u].re += __shfl_xor(s[u].re, off);
      s[u].im += __shfl_xor(s[u].im, off);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int u = 0; u < kFuseK; ++u) red[wv][u] = s[u];
  }
  __syncthreads();
  if ((int)threadIdx.x < min(kp1, kFuseK)) {
    const int u = threadIdx.x;
    cplx t = red[0][u];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      t.re += red[q][u].re;
      t.im += red[q][u].im;
    }
    partial[((size_t)blockIdx.x * ps + u) * nrhs + c] = t;
  }
}

// A HIP event, destroyed with its owner.
struct OwnedEvent {
  hipEvent_t e = nullptr;
  OwnedEvent() = default;
  OwnedEvent(const OwnedEvent&) = delete;
  OwnedEvent& operator=(const OwnedEvent&) = delete;
  ~OwnedEvent() {
    if (e) (void)hipEventDestroy(e);
  }
};

// Pinned host memory lent by the context for the duration of one solve.
struct PinnedLoan {
  dp_ctx* c = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  PinnedLoan() = default;
  PinnedLoan(const PinnedLoan&) = delete;
  PinnedLoan& operator=(const PinnedLoan&) = delete;
  ~PinnedLoan() {
    if (p) pinned_return(c, p, bytes);
  }
};

// Wait for `e` without holding a core: poll it, yielding the thread between
// polls, for at most `spin_us` microseconds (a short expected wait), then
// block on it (the event is created with hipEventBlockingSync).
static int wait_event(hipEvent_t e, int spin_us) {
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    const hipError_t q = hipEventQuery(e);
    if (q == hipSuccess) return DP_OK;
    if (q != hipErrorNotReady) DP_HIP(q);
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(spin_us)) break;
    std::this_thread::yield();
  }
  DP_HIP(hipEventSynchronize(e));
  return DP_OK;
}

// out[i * nrhs + c] = sum_bx partial[(bx * ps + i) * nrhs + c] for i <= *kd
// (fixed order)
__global__ void gram_reduce(const cplx* __restrict__ partial, int nbx, int ps, int nrhs, const int* kd, cplx* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (*kd + 1) * nrhs) return;
  cplx s = {0.0, 0.0};
  for (int b = 0; b < nbx; ++b) {
    const cplx v = partial[(size_t)b * ps * nrhs + t];
    s.re += v.re;
    s.im += v.im;
  }
  out[t] = s;
}

// W[c] -= sum_{i <= *kd} V_i[c] h[i][c]
__global__ void gram_update(const cplx* __restrict__ V, size_t vstride, cplx* __restrict__ W,
                            const cplx* __restrict__ h, int n, int nrhs, const int* kd) {
  const int kp1 = *kd + 1;
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = idx / n;
    cplx acc = W[idx];
    for (int i = 0; i < kp1; ++i) {
      const cplx a = V[i * vstride + idx], b = h[i * nrhs + c];
      acc.re -= a.re * b.re - a.im * b.im;
      acc.im -= a.re * b.im + a.im * b.re;
    }
    W[idx] = acc;
  }
}

// partial[bx * nrhs + c] = sum |W[c]|^2 over the rows of block bx
__global__ __launch_bounds__(256) void col_norm2(const cplx* __restrict__ W, int n, int nrhs, double* partial) {
  __shared__ double red[256];
  const int c = blockIdx.y;
  const int j0 = blockIdx.x * kDotRows;
  const int j1 = min(n, j0 + kDotRows);
  double s = 0.0;
  for (int j = j0 + threadIdx.x; j < j1; j += 256) {
    const cplx a = W[(size_t)c * n + j];
    s = fma(a.re, a.re, fma(a.im, a.im, s));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nrhs + c] = red[0];
}

__global__ void norm_reduce(const double* __restrict__ partial, int nbx, int nrhs, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double s = 0.0;
  for (int b = 0; b < nbx; ++b) s += partial[(size_t)b * nrhs + c];
  out[c] = s;
}

// Y[c] = X[c] * s[c], exactly zero where s[c] == 0
__global__ void scale_cols(const cplx* __restrict__ X, cplx* __restrict__ Y, const double* __restrict__ s, int n,
                           int nrhs) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const double f = s[idx / n];
    const cplx a = X[idx];
    Y[idx] = f != 0.0 ? cplx{a.re * f, a.im * f} : cplx{0.0, 0.0};
  }
}

// The next basis vector V_{k+1}[c] = W[c] * s[c] (k = *kd), exactly zero for
// a stopped column
__global__ void scale_next(const cplx* __restrict__ W, cplx* __restrict__ V, size_t vstride,
                           const double* __restrict__ s, int n, int nrhs, const int* kd) {
  cplx* Vn = V + (size_t)(*kd + 1) * vstride;
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const double f = s[idx / n];
    const cplx a = W[idx];
    Vn[idx] = f != 0.0 ? cplx{a.re * f, a.im * f} : cplx{0.0, 0.0};
  }
}

__global__ void bump_step(int* kd) { *kd += 1; }

// X[c] += sum_{i < kc[c]} Z_i[c] y[i][c]
__global__ void combine(const cplx* __restrict__ Z, size_t zstride, cplx* __restrict__ X,
                        const cplx* __restrict__ y, const int* __restrict__ kc, int n, int nrhs) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = idx / n;
    const int k = kc[c];
    cplx acc = X[idx];
    for (int i = 0; i < k; ++i) {
      const cplx a = Z[i * zstride + idx], b = y[i * nrhs + c];
      acc.re += a.re * b.re - a.im * b.im;
      acc.im += a.re * b.im + a.im * b.re;
    }
    X[idx] = acc;
  }
}

// R = F - AX
__global__ void sub_from(const cplx* __restrict__ F, cplx* __restrict__ R, size_t tot) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const cplx a = F[idx], b = R[idx];
    R[idx] = {a.re - b.re, a.im - b.im};
  }
}

static int g1(size_t tot) {
  size_t g = (tot + 255) / 256;
  return (int)(g > 8192 ? 8192 : (g ? g : 1));
}

__global__ void copy16(const uint4* __restrict__ a, uint4* __restrict__ b, size_t tot) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < tot; q += (size_t)gridDim.x * blockDim.x)
    b[q] = a[q];
}

int dev_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return DP_OK;
  const size_t tot = bytes / 16;
  copy16<<<g1(tot), 256, 0, st>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst), tot);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// ------------------------------------------------ rotation state of a cycle
// Device state of the per-column least-squares problems.  The first part
// (the cycle block: residual estimates, scales, norms and flags) is uploaded
// at the start of a cycle and copied back after every step; it is followed by
// the rotated Hessenberg columns, the rotations and g.
struct CycleState {
  double* est;    // [c] |g_{k+1}| / ||f_c|| after the last step
  double* scl;    // [c] 1/h_{k+1,k} for the next basis vector; 0 for a stopped column
  double* fn;     // [c] ||f_c||
  double* tol;    // [0] stopping tolerance of the estimates
  int* act;       // [c] 1 while the column iterates in this cycle
  int* conv;      // [c] stopped because the estimate met tol (or on breakdown)
  int* its;       // [c] Arnoldi steps over all cycles
  int* kc;        // [c] steps of this cycle
  int* k;         // [0] index of the next step of the cycle
  int* max_iters; // [0]
  cplx* R;        // [(j (m + 1) + i) nrhs + c]: column j of the triangular factor
  cplx* cs;       // [i nrhs + c]: Givens rotation i, [[conj c, conj s], [-s, c]]
  cplx* sn;
  cplx* g;        // [i nrhs + c], i <= m
};

struct CycleLayout {
  size_t est, scl, fn, tol, act, conv, its, kc, k, maxit, block, R, cs, sn, g, total;
};

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

static CycleLayout cycle_layout(int nrhs, int m) {
  CycleLayout L;
  size_t o = 0;
  L.est = o;
  o += 8 * (size_t)nrhs;
  L.scl = o;
  o += 8 * (size_t)nrhs;
  L.fn = o;
  o += 8 * (size_t)nrhs;
  L.tol = o;
  o += 8;
  L.act = o;
  o += 4 * (size_t)nrhs;
  L.conv = o;
  o += 4 * (size_t)nrhs;
  L.its = o;
  o += 4 * (size_t)nrhs;
  L.kc = o;
  o += 4 * (size_t)nrhs;
  L.k = o;
  o += 4;
  L.maxit = o;
  o += 4;
  L.block = o;
  o = up256(o);
  L.R = o;
  o += (size_t)m * (m + 1) * nrhs * sizeof(cplx);
  L.cs = o;
  o += (size_t)m * nrhs * sizeof(cplx);
  L.sn = o;
  o += (size_t)m * nrhs * sizeof(cplx);
  L.g = o;
  o += (size_t)(m + 1) * nrhs * sizeof(cplx);
  L.total = o;
  return L;
}

static CycleState cycle_state(void* base, const CycleLayout& L) {
  char* b = static_cast<char*>(base);
  CycleState s;
  s.est = reinterpret_cast<double*>(b + L.est);
  s.scl = reinterpret_cast<double*>(b + L.scl);
  s.fn = reinterpret_cast<double*>(b + L.fn);
  s.tol = reinterpret_cast<double*>(b + L.tol);
  s.act = reinterpret_cast<int*>(b + L.act);
  s.conv = reinterpret_cast<int*>(b + L.conv);
  s.its = reinterpret_cast<int*>(b + L.its);
  s.kc = reinterpret_cast<int*>(b + L.kc);
  s.k = reinterpret_cast<int*>(b + L.k);
  s.max_iters = reinterpret_cast<int*>(b + L.maxit);
  s.R = reinterpret_cast<cplx*>(b + L.R);
  s.cs = reinterpret_cast<cplx*>(b + L.cs);
  s.sn = reinterpret_cast<cplx*>(b + L.sn);
  s.g = reinterpret_cast<cplx*>(b + L.g);
  return s;
}

__device__ __forceinline__ cplx cmul_(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cconj_mul(cplx a, cplx b) {  // conj(a) b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// After the orthogonalisation of step k = *s.k: the new Hessenberg column
// h_i = h1_i + h2_i (i <= k) and h_{k+1} = ||w|| of column c = blockIdx.x;
// the previous rotations, the new one, g and the stopping test (Sec. 3: a
// column stops when its relative residual estimate meets tol).  The column's
// data go through LDS (the block loads them in parallel); one thread applies
// the rotations in order.  Stopped columns keep their state.
__global__ __launch_bounds__(64) void arnoldi_rotate(const cplx* __restrict__ h1, const cplx* __restrict__ h2,
                                                     const double* __restrict__ nrm2, CycleState s, int nrhs, int m) {
  extern __shared__ cplx lds[];  // h[0..k], cs[0..k-1], sn[0..k-1]
  const int c = blockIdx.x;
  const int k = *s.k;
  if (!s.act[c]) {
    if (threadIdx.x == 0) s.scl[c] = 0.0;
    return;
  }
  cplx* hh = lds;
  cplx* cc = lds + (k + 1);
  cplx* ss = cc + k;
  for (int i = threadIdx.x; i <= k; i += 64) {
    const cplx a = h1[(size_t)i * nrhs + c], b = h2[(size_t)i * nrhs + c];
    hh[i] = {a.re + b.re, a.im + b.im};
  }
  for (int i = threadIdx.x; i < k; i += 64) {
    cc[i] = s.cs[(size_t)i * nrhs + c];
    ss[i] = s.sn[(size_t)i * nrhs + c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(nrm2[c]);
    cplx cur = hh[0];
    for (int i = 0; i < k; ++i) {
      const cplx ci = cc[i], si = ss[i], nx = hh[i + 1];
      const cplx t0 = cconj_mul(ci, cur), t1 = cconj_mul(si, nx);
      const cplx u0 = cmul_(si, cur), u1 = cmul_(ci, nx);
      hh[i] = {t0.re + t1.re, t0.im + t1.im};
      cur = {u1.re - u0.re, u1.im - u0.im};
    }
    const double den = sqrt(cur.re * cur.re + cur.im * cur.im + hn * hn);
    const cplx ck = den > 0.0 ? cplx{cur.re / den, cur.im / den} : cplx{1.0, 0.0};
    const cplx sk = den > 0.0 ? cplx{hn / den, 0.0} : cplx{0.0, 0.0};
    hh[k] = {den, 0.0};
    s.cs[(size_t)k * nrhs + c] = ck;
    s.sn[(size_t)k * nrhs + c] = sk;
    const cplx gk = s.g[(size_t)k * nrhs + c];
    const cplx gn = cmul_(sk, gk);
    s.g[(size_t)(k + 1) * nrhs + c] = {-gn.re, -gn.im};
    s.g[(size_t)k * nrhs + c] = cconj_mul(ck, gk);
    const double est = sqrt(gn.re * gn.re + gn.im * gn.im) / s.fn[c];
    const int its = s.its[c] + 1;
    s.its[c] = its;
    s.kc[c] = k + 1;
    s.est[c] = est;
    const bool met = est <= *s.tol || hn == 0.0;
    if (met || its >= *s.max_iters) {
      s.act[c] = 0;
      s.conv[c] = met ? 1 : 0;
      s.scl[c] = 0.0;
    } else {
      s.scl[c] = 1.0 / hn;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= k; i += 64) s.R[((size_t)k * (m + 1) + i) * nrhs + c] = hh[i];
}

// End of a cycle: y = R^{-1} g for column c = blockIdx.x over its kc[c]
// steps (back substitution by columns of R, the running right-hand side in
// LDS), y[i][c] = 0 for kc[c] <= i < m.
__global__ __launch_bounds__(64) void arnoldi_solve(CycleState s, cplx* __restrict__ y, int nrhs, int m) {
  extern __shared__ cplx lds[];  // right-hand side, then the solution
  const int c = blockIdx.x;
  const int kk = s.kc[c];
  cplx* r = lds;
  for (int i = threadIdx.x; i < kk; i += 64) r[i] = s.g[(size_t)i * nrhs + c];
  __syncthreads();
  for (int i = kk - 1; i >= 0; --i) {
    const double d = s.R[((size_t)i * (m + 1) + i) * nrhs + c].re;  // real after the rotation
    const cplx yi = d != 0.0 ? cplx{r[i].re / d, r[i].im / d} : cplx{0.0, 0.0};
    for (int j = threadIdx.x; j < i; j += 64) {
      const cplx a = s.R[((size_t)i * (m + 1) + j) * nrhs + c];
      const cplx t = cmul_(a, yi);
      r[j] = {r[j].re - t.re, r[j].im - t.im};
    }
    __syncthreads();
    if (threadIdx.x == 0) r[i] = yi;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < m; i += 64) y[(size_t)i * nrhs + c] = i < kk ? r[i] : cplx{0.0, 0.0};
}

// Column norms ||W_c||_2 into host vector out.
static int norms(dp_problem* p, const cplx* W, int nrhs, DevBuf& part, std::vector<double>& out) {
  const int n = (int)p->n;
  const int nbx = (n + kDotRows - 1) / kDotRows;
  hipStream_t st = p->ctx->stream;
  DP_TRY(part.reserve(((size_t)nbx + 1) * nrhs * sizeof(double)));
  double* pp = part.as<double>();
  col_norm2<<<dim3(nbx, nrhs), 256, 0, st>>>(W, n, nrhs, pp);
  norm_reduce<<<(nrhs + 63) / 64, 64, 0, st>>>(pp, nbx, nrhs, pp + (size_t)nbx * nrhs);
  out.resize(nrhs);
  DP_HIP(hipMemcpyAsync(out.data(), pp + (size_t)nbx * nrhs, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  for (auto& v : out) v = sqrt(v);
  return DP_OK;
}

// The device part of an Arnoldi step after w = A P v_k: CGS2 against
// V_0..V_k, the norm of w, the rotation update and the next basis vector;
// then the step index advances.  `fuse`: basis sizes up to kFuseK.
struct Tail {
  cplx *V, *W, *part, *h1, *h2;
  double* nrm;
  CycleState s;
  size_t blk;
  int n, nrhs, m, nbx;
};

static void launch_tail(const Tail& t, bool fuse, hipStream_t st) {
  const int ps = t.m + 1;
  const int rg = (ps * t.nrhs + 255) / 256;
  const dim3 gd(t.nbx, t.nrhs);
  gram_dots<<<gd, 256, 0, st>>>(t.V, t.blk, t.W, t.n, t.nrhs, t.s.k, ps, t.part);
  gram_reduce<<<rg, 256, 0, st>>>(t.part, t.nbx, ps, t.nrhs, t.s.k, t.h1);
  if (fuse) {
    gram_update_dots<<<gd, 256, 0, st>>>(t.V, t.blk, t.W, t.h1, t.n, t.nrhs, t.s.k, ps, t.part);
  } else {
    gram_update<<<g1(t.blk), 256, 0, st>>>(t.V, t.blk, t.W, t.h1, t.n, t.nrhs, t.s.k);
    gram_dots<<<gd, 256, 0, st>>>(t.V, t.blk, t.W, t.n, t.nrhs, t.s.k, ps, t.part);
  }
  gram_reduce<<<rg, 256, 0, st>>>(t.part, t.nbx, ps, t.nrhs, t.s.k, t.h2);
  gram_update<<<g1(t.blk), 256, 0, st>>>(t.V, t.blk, t.W, t.h2, t.n, t.nrhs, t.s.k);
  double* pp = reinterpret_cast<double*>(t.part);
  col_norm2<<<gd, 256, 0, st>>>(t.W, t.n, t.nrhs, pp);
  norm_reduce<<<(t.nrhs + 63) / 64, 64, 0, st>>>(pp, t.nbx, t.nrhs, t.nrm);
  arnoldi_rotate<<<t.nrhs, 64, (3 * (size_t)t.m + 1) * sizeof(cplx), st>>>(t.h1, t.h2, t.nrm, t.s, t.nrhs, t.m);
  scale_next<<<g1(t.blk), 256, 0, st>>>(t.W, t.V, t.blk, t.s.scl, t.n, t.nrhs, t.s.k);
  bump_step<<<1, 1, 0, st>>>(t.s.k);
}

// The two executable graphs of launch_tail for this problem's current
// workspaces, captured on first use (again when a workspace moved or the
// sizes changed).  Returns false when capture is not possible here; the
// caller then launches the kernels directly.
static bool tail_graphs(dp_problem* p, const Tail& t) {
  if (!p->kgraph_ok) return false;
  const std::vector<void*> sig = {t.V, t.W, t.part, t.h1, t.s.est, (void*)(intptr_t)t.n, (void*)(intptr_t)t.nrhs,
                                  (void*)(intptr_t)t.m};
  if (p->kgraph[0] && sig == p->kgraph_sig) return true;
  for (auto& g : p->kgraph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  hipStream_t st = p->ctx->stream;
  for (int v = 0; v < 2; ++v) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    bool ok;
    {
      CaptureScope excl;  // no stream-ordered allocation in any thread until instantiated
      ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        launch_tail(t, v == 0, st);
        ok = hipStreamEndCapture(st, &g) == hipSuccess && g;
      }
      ok = ok && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ok) {
      if (x) (void)hipGraphExecDestroy(x);
      for (auto& e : p->kgraph) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
      p->kgraph_ok = false;
      return false;
    }
    p->kgraph[v] = x;
  }
  p->kgraph_sig = sig;
  return true;
}

void krylov_graphs_destroy(dp_problem* p) {
  for (auto& g : p->kgraph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  p->kgraph_sig.clear();
}

// Restarted (flexible) GMRES with operator precision `prec` (0 FP64, 1 mixed)
// from x0 = 0; the residual checks at restarts use the same operator.  With
// `trust_estimate` (the correction solves of the refinement) a column whose
// Arnoldi residual estimate meets tol is final without a true-residual check:
// the single-precision operator's own rounding can hold its true residual just
// above a tight inner tolerance, and the FP64 residual of the outer step is the
// real test.
static int gmres_core(dp_problem* p, int nrhs, const cplx* F, cplx* X, const dp_solve_opts* o, int prec,
                      bool trust_estimate, dp_solve_info* info, int64_t* iters_out, double* relres_out) {
  const auto t0 = std::chrono::steady_clock::now();
  const int n = (int)p->n;
  const double tol = o->tol;
  const int m = o->restart;
  const bool pre = o->use_precond != 0;
  hipStream_t st = p->ctx->stream;
  const size_t blk = (size_t)n * nrhs;

  DevBuf &V = p->krylov_ws[0], &Zb = p->krylov_ws[1], &W = p->krylov_ws[2], &R = p->krylov_ws[3],
         &part = p->krylov_ws[4], &small = p->krylov_ws[5], &kst = p->krylov_ws[6];
  DP_TRY(V.reserve((m + 1) * blk * sizeof(cplx)));
  if (pre) DP_TRY(Zb.reserve(m * blk * sizeof(cplx)));
  DP_TRY(W.reserve(blk * sizeof(cplx)));
  DP_TRY(R.reserve(blk * sizeof(cplx)));
  const int nbx = (n + kDotRows - 1) / kDotRows;
  DP_TRY(part.reserve((size_t)nbx * (m + 1) * nrhs * sizeof(cplx) + 64));
  // small: h1 (m+1)*nrhs, h2 (m+1)*nrhs, norm^2 nrhs (as cplx slots), y m*nrhs
  const size_t hsz = (size_t)(m + 1) * nrhs;
  DP_TRY(small.reserve((2 * hsz + (size_t)nrhs + (size_t)m * nrhs) * sizeof(cplx)));
  const CycleLayout L = cycle_layout(nrhs, m);
  DP_TRY(kst.reserve(L.total));
  cplx* h1 = small.as<cplx>();
  cplx* h2 = h1 + hsz;
  double* nrm = reinterpret_cast<double*>(h2 + hsz);
  cplx* ydev = h2 + hsz + nrhs;
  cplx* Vp = V.as<cplx>();
  cplx* Zp = pre ? Zb.as<cplx>() : Vp;
  cplx* Wp = W.as<cplx>();
  cplx* Rp = R.as<cplx>();
  const CycleState ks = cycle_state(kst.p, L);
  const Tail tail = {Vp, Wp, part.as<cplx>(), h1, h2, nrm, ks, blk, n, nrhs, m, nbx};
  const bool graphs = !o->eager && tail_graphs(p, tail);
  // test hook: queue every step without the prediction, so that steps queued
  // after the last column stopped do occur (they must change nothing)
  const char* aq = std::getenv("DIRPREC_TEST_ALWAYS_QUEUE");
  const bool always_queue = aq && aq[0] == '1';

  SweepClock tm, ta;  // matrix-vector products and applies of the queued steps
  int64_t matvecs = 0, applies = 0;

  std::vector<double> fn, beta;
  DP_TRY(norms(p, F, nrhs, part, fn));
  DP_HIP(hipMemsetAsync(X, 0, blk * sizeof(cplx), st));
  DP_TRY(dev_copy(Rp, F, blk * sizeof(cplx), st));
  beta = fn;
  std::vector<char> done(nrhs, 0);
  std::vector<int64_t> its(nrhs, 0);
  std::vector<double> rel(nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c) {
    rel[c] = fn[c] > 0 ? 1.0 : 0.0;
    if (fn[c] == 0) done[c] = 1;
  }
  OwnedEvent ev[2];  // after the state readback of even / odd steps
  for (auto& e : ev) DP_HIP(hipEventCreateWithFlags(&e.e, hipEventDisableTiming | hipEventBlockingSync));
  // pinned host memory: two readback slots of the cycle block, the upload
  // block and the first row of g
  const size_t bb = up256(L.block);
  PinnedLoan hpin;
  hpin.c = p->ctx;
  DP_TRY(pinned_borrow(p->ctx, 3 * bb + (size_t)nrhs * sizeof(cplx), &hpin.p, &hpin.bytes));
  char* hb = static_cast<char*>(hpin.p);
  const CycleState slot[2] = {cycle_state(hb, L), cycle_state(hb + bb, L)};
  const CycleState up = cycle_state(hb + 2 * bb, L);
  cplx* g0 = reinterpret_cast<cplx*>(hb + 3 * bb);
  std::vector<double> e_last(nrhs), e_prev(nrhs);
  std::vector<int> its_last(nrhs), act_last(nrhs);
  int rc = DP_OK;

  while (true) {
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      const bool a = !done[c] && its[c] < o->max_iters;
      any |= a;
      up.est[c] = rel[c];
      up.scl[c] = a ? 1.0 / beta[c] : 0.0;
      up.fn[c] = fn[c];
      up.act[c] = a;
      up.conv[c] = 0;
      up.its[c] = (int)its[c];
      up.kc[c] = 0;
      g0[c] = a ? cplx{beta[c], 0.0} : cplx{0.0, 0.0};
      e_last[c] = e_prev[c] = rel[c];
      its_last[c] = (int)its[c];
      act_last[c] = a;
    }
    if (!any) break;
    *up.tol = tol;
    *up.k = 0;
    *up.max_iters = o->max_iters;
    DP_HIP(hipMemcpyAsync(ks.est, up.est, L.block, hipMemcpyHostToDevice, st));
    DP_HIP(hipMemcpyAsync(ks.g, g0, (size_t)nrhs * sizeof(cplx), hipMemcpyHostToDevice, st));
    scale_cols<<<g1(blk), 256, 0, st>>>(Rp, Vp, ks.scl, n, nrhs);
    int steps = 0;       // useful steps queued in this cycle
    int known = -1;      // last step whose state the host has read
    int last_slot = -1;  // slot of the last queued step's readback
    for (int k = 0; k < m; ++k) {
      const size_t mk_tm = tm.used, mk_ta = ta.used, mk_c = p->clock.used, mk_c32 = p->clock32.used;
      cplx* vk = Vp + k * blk;
      cplx* zk = Zp + k * blk;
      if (pre) {
        ta.start(st);
        DP_TRY(precond_apply(p, nrhs, vk, zk, prec));
        ta.stop(st);
      }
      tm.start(st);
      p->sweep_guard = ks.act;
      p->sweep_guard_n = nrhs;
      const int mrc = matvec(p, nrhs, zk, Wp, prec);
      p->sweep_guard = nullptr;
      p->sweep_guard_n = 0;
      DP_TRY(mrc);
      tm.stop(st);
      const bool fuse = k + 1 <= kFuseK;
      if (graphs) DP_HIP(hipGraphLaunch(p->kgraph[fuse ? 0 : 1], st));
      else launch_tail(tail, fuse, st);
      DP_HIP(hipGetLastError());
      DP_HIP(hipMemcpyAsync(slot[k & 1].est, ks.est, L.block, hipMemcpyDeviceToHost, st));
      DP_HIP(hipEventRecord(ev[k & 1].e, st));
      last_slot = k & 1;
      steps = k + 1;
      // the state after step k - 1 (normally complete while step k runs)
      if (k >= 1 && known < k - 1) {
        DP_TRY(wait_event(ev[(k - 1) & 1].e, 0));
        known = k - 1;
        const CycleState& sl = slot[(k - 1) & 1];
        bool run = false;
        for (int c = 0; c < nrhs; ++c) {
          run |= sl.act[c] != 0;
          if (act_last[c]) {
            e_prev[c] = e_last[c];
            e_last[c] = sl.est[c];
          }
          its_last[c] = sl.its[c];
          act_last[c] = sl.act[c];
        }
        if (!run) {
          // step k was queued after every column stopped: it changed no
          // state; drop its timings
          tm.used = mk_tm;
          ta.used = mk_ta;
          p->clock.used = mk_c;
          p->clock32.used = mk_c32;
          steps = k;
          break;
        }
      }
      if (k + 1 >= m) break;
      // May step k stop the last running columns?  Predict each column's
      // estimate after step k from its last two (a geometric rate, at most
      // 20x per step); if no column is sure to keep running, wait for step k
      // before queuing step k + 1.
      bool sure = always_queue;
      for (int c = 0; c < nrhs && !sure; ++c) {
        if (!act_last[c]) continue;
        double r = e_prev[c] > 0.0 ? e_last[c] / e_prev[c] : 1.0;
        r = r > 1.0 ? 1.0 : (r < 0.05 ? 0.05 : r);
        const bool more_steps = its_last[c] + (k - known) < o->max_iters;
        sure = more_steps && e_last[c] * r > 8.0 * tol;
      }
      if (!sure) {
        DP_TRY(wait_event(ev[k & 1].e, 2000));
        known = k;
        const CycleState& sl = slot[k & 1];
        bool run = false;
        for (int c = 0; c < nrhs; ++c) {
          run |= sl.act[c] != 0;
          if (act_last[c]) {
            e_prev[c] = e_last[c];
            e_last[c] = sl.est[c];
          }
          its_last[c] = sl.its[c];
          act_last[c] = sl.act[c];
        }
        if (!run) break;
      }
    }
    matvecs += steps;
    applies += pre ? steps : 0;
    // y = R^{-1} g per column, X += Z y
    arnoldi_solve<<<nrhs, 64, (size_t)m * sizeof(cplx), st>>>(ks, ydev, nrhs, m);
    combine<<<g1(blk), 256, 0, st>>>(Zp, blk, X, ydev, ks.kc, n, nrhs);
    DP_HIP(hipGetLastError());
    DP_TRY(wait_event(ev[last_slot].e, 0));
    const CycleState& fin = slot[last_slot];
    std::vector<char> conv_est(nrhs, 0);
    for (int c = 0; c < nrhs; ++c) {
      if (done[c] || its[c] >= o->max_iters) continue;
      its[c] = fin.its[c];
      rel[c] = fin.est[c];
      conv_est[c] = fin.conv[c] != 0;
    }
    if (trust_estimate) {
      bool more = false;
      for (int c = 0; c < nrhs; ++c) {
        if (conv_est[c]) done[c] = 1;
        more |= !done[c] && its[c] < o->max_iters;
      }
      if (!more) break;
    }
    // true residual
    tm.start(st);
    DP_TRY(matvec(p, nrhs, X, Rp, prec));
    tm.stop(st);
    ++matvecs;
    sub_from<<<g1(blk), 256, 0, st>>>(F, Rp, blk);
    DP_TRY(norms(p, Rp, nrhs, part, beta));
    bool cont = false;
    for (int c = 0; c < nrhs; ++c) {
      if (done[c]) continue;
      rel[c] = fn[c] > 0 ? beta[c] / fn[c] : 0.0;
      if (rel[c] <= tol) done[c] = 1;
      else if (its[c] < o->max_iters) cont = true;
    }
    if (!cont) break;
  }
  double rmax = 0;
  int64_t imax = 0;
  for (int c = 0; c < nrhs; ++c) {
    if (!done[c]) rc = DP_ENOCONV;
    rmax = rel[c] > rmax ? rel[c] : rmax;
    imax = its[c] > imax ? its[c] : imax;
    if (iters_out) iters_out[c] = its[c];
    if (relres_out) relres_out[c] = rel[c];
  }
  DP_HIP(hipStreamSynchronize(st));
  tm.collect();
  ta.collect();
  p->clock.collect();
  p->clock32.collect();
  if (info) {
    info->iters_max = imax;
    info->matvecs = matvecs;
    info->applies = applies;
    info->relres_max = rmax;
    info->t_matvec = tm.seconds;
    info->t_apply = ta.seconds;
    info->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_krylov = info->t_total - tm.seconds - ta.seconds;
    info->sweep_launches = p->clock.launches;
    info->t_sweep = p->clock.seconds;
    info->refinements = 0;
    info->matvecs_fp32 = prec ? matvecs : 0;
    info->sweep_launches_fp32 = p->clock32.launches;
    info->t_sweep_fp32 = p->clock32.seconds;
  }
  tm.destroy();
  ta.destroy();
  return rc;  // the workspaces stay with the problem
}

// out[c] = F[c] - R[c] for columns with keep[c] != 0, else 0
__global__ void residual_cols(const cplx* __restrict__ F, cplx* __restrict__ R, const double* __restrict__ keep,
                              int n, int nrhs) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const cplx a = F[idx], b = R[idx];
    R[idx] = keep[idx / n] != 0.0 ? cplx{a.re - b.re, a.im - b.im} : cplx{0.0, 0.0};
  }
}

// X += D
__global__ void add_into(cplx* __restrict__ X, const cplx* __restrict__ D, size_t tot) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const cplx a = X[idx], b = D[idx];
    X[idx] = {a.re + b.re, a.im + b.im};
  }
}

int solve(dp_problem* p, int nrhs, const cplx* F, cplx* X, const dp_solve_opts* o, dp_solve_info* info,
          int64_t* iters_out, double* relres_out) {
  p->clock.reset();
  p->clock32.reset();
  if (o->precision == DP_PREC_FP64) return gmres_core(p, nrhs, F, X, o, 0, false, info, iters_out, relres_out);
  // Mixed precision: q_{k+1} = q_k + GMRES_32(f - A q_k), residuals in FP64.
  const auto t0 = std::chrono::steady_clock::now();
  const int n = (int)p->n;
  hipStream_t st = p->ctx->stream;
  const size_t blk = (size_t)n * nrhs;
  DevBuf &R = p->refine_ws[0], &D = p->refine_ws[1], &part = p->refine_ws[2], &keep = p->refine_ws[3];
  DP_TRY(R.reserve(blk * sizeof(cplx)));
  DP_TRY(D.reserve(blk * sizeof(cplx)));
  DP_TRY(keep.reserve(nrhs * sizeof(double)));
  std::vector<double> fn, rn;
  DP_TRY(norms(p, F, nrhs, part, fn));
  DP_HIP(hipMemsetAsync(X, 0, blk * sizeof(cplx), st));
  DP_TRY(dev_copy(R.p, F, blk * sizeof(cplx), st));
  std::vector<int64_t> its(nrhs, 0), its_in(nrhs);
  std::vector<double> rel(nrhs, 1.0), rel_in(nrhs), kv(nrhs);
  for (int c = 0; c < nrhs; ++c) rel[c] = fn[c] > 0 ? 1.0 : 0.0;
  dp_solve_opts oi = *o;
  oi.tol = o->inner_tol;
  int64_t mv = 0, mv32 = 0, ap = 0, outer = 0;
  double t_mv = 0, t_ap = 0;
  SweepClock tm;  // the FP64 residual products
  int rc = DP_OK;
  const int max_outer = 12;
  while (true) {
    bool any = false;
    int64_t left = o->max_iters;
    for (int c = 0; c < nrhs; ++c)
      if (rel[c] > o->tol) {
        any = true;
        left = std::min<int64_t>(left, o->max_iters - its[c]);
      }
    if (!any) break;
    if (outer >= max_outer || left <= 0) {
      rc = DP_ENOCONV;
      break;
    }
    oi.max_iters = (int)std::max<int64_t>(1, left);
    // A column at FP64 residual rel needs its correction solve to reduce the
    // residual by tol/rel only; ask for 0.3 of that for the worst column (its
    // FP64 residual then ends near 0.3 tol, and a column that still misses tol
    // gets one more refinement), and never less than inner_tol (the first
    // step, rel = 1, gets inner_tol).
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c)
      if (rel[c] > o->tol) worst = std::max(worst, rel[c]);
    oi.tol = std::max(o->inner_tol, worst > 0.0 ? 0.3 * o->tol / worst : o->inner_tol);
    dp_solve_info ii;
    int r = gmres_core(p, nrhs, R.as<cplx>(), D.as<cplx>(), &oi, 1, true, &ii, its_in.data(), rel_in.data());
    if (r < 0) return r;
    for (int c = 0; c < nrhs; ++c) its[c] += its_in[c];
    mv += ii.matvecs;
    mv32 += ii.matvecs;
    ap += ii.applies;
    t_mv += ii.t_matvec;
    t_ap += ii.t_apply;
    ++outer;
    const size_t g = (blk + 255) / 256;
    add_into<<<(int)(g > 8192 ? 8192 : g), 256, 0, st>>>(X, D.as<cplx>(), blk);
    // R = f - A X in FP64 (converged columns get zero right-hand sides)
    tm.start(st);
    DP_TRY(matvec(p, nrhs, X, R.as<cplx>(), 0));
    tm.stop(st);
    ++mv;
    for (int c = 0; c < nrhs; ++c) kv[c] = 1.0;
    DP_HIP(hipMemcpyAsync(keep.p, kv.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    residual_cols<<<(int)(g > 8192 ? 8192 : g), 256, 0, st>>>(F, R.as<cplx>(), keep.as<double>(), n, nrhs);
    DP_TRY(norms(p, R.as<cplx>(), nrhs, part, rn));
    tm.collect();
    p->clock.collect();
    p->clock32.collect();
    bool zero_any = false;
    for (int c = 0; c < nrhs; ++c) {
      rel[c] = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
      kv[c] = rel[c] > o->tol ? 1.0 : 0.0;
      zero_any |= kv[c] == 0.0;
    }
    if (zero_any) {
      DP_HIP(hipMemcpyAsync(keep.p, kv.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
      // zero the residual columns that already meet tol (their corrections vanish)
      scale_cols<<<(int)(g > 8192 ? 8192 : g), 256, 0, st>>>(R.as<cplx>(), R.as<cplx>(), keep.as<double>(), n,
                                                             nrhs);
    }
  }
  DP_HIP(hipStreamSynchronize(st));
  double rmax = 0;
  int64_t imax = 0;
  for (int c = 0; c < nrhs; ++c) {
    rmax = std::max(rmax, rel[c]);
    imax = std::max(imax, its[c]);
    if (iters_out) iters_out[c] = its[c];
    if (relres_out) relres_out[c] = rel[c];
  }
  if (info) {
    info->iters_max = imax;
    info->matvecs = mv;
    info->applies = ap;
    info->relres_max = rmax;
    info->t_matvec = t_mv + tm.seconds;
    info->t_apply = t_ap;
    info->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_krylov = info->t_total - info->t_matvec - t_ap;
    info->sweep_launches = p->clock.launches;
    info->t_sweep = p->clock.seconds;
    info->refinements = outer;
    info->matvecs_fp32 = mv32;
    info->sweep_launches_fp32 = p->clock32.launches;
    info->t_sweep_fp32 = p->clock32.seconds;
  }
  tm.destroy();
  return rc;  // the workspaces stay with the problem
}

}  // namespace dp
