// Restarted GMRES for A q = f with nrhs independent columns (Sec. 3: GMRES,
// restart 80, relative tolerance).  Right preconditioning is done in the
// flexible form: z_k = P v_k is stored and the iterate is x = x0 + Z y, so no
// extra preconditioner application is needed and the residual is the true
// one.  Arnoldi uses classical Gram-Schmidt applied twice (CGS2) so that each
// step is two block dot-product / update sweeps over the basis; the small
// Hessenberg least-squares problems (Givens rotations) live on the host, one
// D2H copy of (k+2) coefficients per column per step.  A column stops its
// cycle when its Givens residual estimate reaches tol; at each restart the
// true residual f - A x is recomputed and decides convergence.
#include <chrono>
#include <thread>
#include <complex>
#include <cstring>
#include <vector>

#include "dp_internal.hpp"

namespace dp {

using zc = std::complex<double>;

constexpr int kDotRows = 2048;

// partial[(bx * kp1 + i) * nrhs + c] = sum_{rows of block bx} conj(V_i[c]) W[c]
__global__ __launch_bounds__(256) void gram_dots(const cplx* __restrict__ V, size_t vstride,
                                                 const cplx* __restrict__ W, int n, int nrhs, int kp1,
                                                 cplx* __restrict__ partial) {
  // eight basis vectors per pass over the rows; each sum is reduced within
  // its wave by a fixed butterfly, then over the four waves in order
  constexpr int G = 8;
  __shared__ cplx red[4][G];
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
      partial[((size_t)blockIdx.x * kp1 + i0 + u) * nrhs + c] = t;
    }
    __syncthreads();
  }
}

// The first projection's update and the second projection's dot products in
// one pass over the basis, for kp1 <= kFuseK: per row, W[c] -= sum_i V_i[c]
// h[i][c] with the row's basis values held in registers, then the partial
// sums conj(V_i[c]) W[c] of the updated row, reduced as in gram_dots.  The
// grid is that of gram_dots.
constexpr int kFuseK = 16;

__global__ __launch_bounds__(256) void gram_update_dots(const cplx* __restrict__ V, size_t vstride,
                                                        cplx* __restrict__ W, const cplx* __restrict__ h, int n,
                                                        int nrhs, int kp1, cplx* __restrict__ partial) {
  __shared__ cplx red[4][kFuseK];
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
  if ((int)threadIdx.x < kp1) {
    const int u = threadIdx.x;
    cplx t = red[0][u];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      t.re += red[q][u].re;
      t.im += red[q][u].im;
    }
    partial[((size_t)blockIdx.x * kp1 + u) * nrhs + c] = t;
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
// polls, for at most `spin_us` microseconds (the short tail of a step), then
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

// out[i * nrhs + c] = sum_bx partial[...]  (fixed order)
__global__ void gram_reduce(const cplx* __restrict__ partial, int nbx, int kp1, int nrhs, cplx* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kp1 * nrhs) return;
  cplx s = {0.0, 0.0};
  for (int b = 0; b < nbx; ++b) {
    const cplx v = partial[(size_t)b * kp1 * nrhs + t];
    s.re += v.re;
    s.im += v.im;
  }
  out[t] = s;
}

// W[c] -= sum_i V_i[c] h[i][c]
__global__ void gram_update(const cplx* __restrict__ V, size_t vstride, cplx* __restrict__ W,
                            const cplx* __restrict__ h, int n, int nrhs, int kp1) {
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

// Y[c] = X[c] * s[c]
__global__ void scale_cols(const cplx* __restrict__ X, cplx* __restrict__ Y, const double* __restrict__ s, int n,
                           int nrhs) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const double f = s[idx / n];
    const cplx a = X[idx];
    Y[idx] = {a.re * f, a.im * f};
  }
}

// X[c] += sum_i Z_i[c] y[i][c]
__global__ void combine(const cplx* __restrict__ Z, size_t zstride, cplx* __restrict__ X,
                        const cplx* __restrict__ y, int n, int nrhs, int k) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = idx / n;
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

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  double acc = 0;
  bool pending = false;
  void init() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  void start(hipStream_t s) { (void)hipEventRecord(a, s); }
  void stop(hipStream_t s) {
    (void)hipEventRecord(b, s);
    pending = true;
  }
  void collect() {
    if (!pending) return;
    float ms = 0;
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    acc += ms * 1e-3;
    pending = false;
  }
  void destroy() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

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
         &part = p->krylov_ws[4], &small = p->krylov_ws[5];
  DP_TRY(V.reserve((m + 1) * blk * sizeof(cplx)));
  if (pre) DP_TRY(Zb.reserve(m * blk * sizeof(cplx)));
  DP_TRY(W.reserve(blk * sizeof(cplx)));
  DP_TRY(R.reserve(blk * sizeof(cplx)));
  const int nbx = (n + kDotRows - 1) / kDotRows;
  DP_TRY(part.reserve((size_t)nbx * (m + 1) * nrhs * sizeof(cplx) + 64));
  // small: h1 (m+1)*nrhs, h2 (m+1)*nrhs, norm^2 nrhs (as cplx slots), scale nrhs, y m*nrhs
  const size_t hsz = (size_t)(m + 1) * nrhs;
  DP_TRY(small.reserve((2 * hsz + 2 * (size_t)nrhs + (size_t)m * nrhs) * sizeof(cplx)));
  cplx* h1 = small.as<cplx>();
  cplx* h2 = h1 + hsz;
  double* nrm = reinterpret_cast<double*>(h2 + hsz);
  double* scl = nrm + nrhs;
  cplx* ydev = reinterpret_cast<cplx*>(scl + nrhs);
  cplx* Vp = V.as<cplx>();
  cplx* Zp = pre ? Zb.as<cplx>() : Vp;
  cplx* Wp = W.as<cplx>();
  cplx* Rp = R.as<cplx>();

  Timer tm, ta;
  tm.init();
  ta.init();
  int64_t matvecs = 0, applies = 0;

  std::vector<double> fn, beta;
  DP_TRY(norms(p, F, nrhs, part, fn));
  DP_HIP(hipMemsetAsync(X, 0, blk * sizeof(cplx), st));
  DP_HIP(hipMemcpyAsync(Rp, F, blk * sizeof(cplx), hipMemcpyDeviceToDevice, st));
  beta = fn;
  std::vector<char> done(nrhs, 0);
  std::vector<int64_t> its(nrhs, 0);
  std::vector<double> rel(nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c) {
    rel[c] = fn[c] > 0 ? 1.0 : 0.0;
    if (fn[c] == 0) done[c] = 1;
  }
  std::vector<zc> H((size_t)(m + 1) * m * nrhs), cs((size_t)m * nrhs), sn((size_t)m * nrhs),
      g((size_t)(m + 1) * nrhs);
  std::vector<int> kc(nrhs);
  std::vector<char> active(nrhs), conv_est(nrhs);
  OwnedEvent ev_mv, ev_rb;  // after each step's matrix-vector product / readback
  DP_HIP(hipEventCreateWithFlags(&ev_mv.e, hipEventDisableTiming | hipEventBlockingSync));
  DP_HIP(hipEventCreateWithFlags(&ev_rb.e, hipEventDisableTiming | hipEventBlockingSync));
  // pinned host copy of h1 | h2 | norm^2 | scale (the layout of `small`):
  // the per-step readback is one asynchronous copy, with no staging through
  // pageable memory
  PinnedLoan hpin;
  hpin.c = p->ctx;
  DP_TRY(pinned_borrow(p->ctx, (2 * hsz + 2 * (size_t)nrhs) * sizeof(cplx), &hpin.p, &hpin.bytes));
  cplx* hbuf = static_cast<cplx*>(hpin.p);
  double* nbuf = reinterpret_cast<double*>(hbuf + 2 * hsz);
  double* sbuf = nbuf + nrhs;
  std::vector<cplx> yh((size_t)m * nrhs);
  int rc = DP_OK;
  auto Hat = [&](int i, int k, int c) -> zc& { return H[((size_t)c * (m + 1) + i) * m + k]; };

  while (true) {
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      active[c] = !done[c] && its[c] < o->max_iters;
      conv_est[c] = 0;
      any |= active[c];
      sbuf[c] = active[c] ? 1.0 / beta[c] : 0.0;
      kc[c] = 0;
      g[(size_t)c * (m + 1)] = active[c] ? zc(beta[c], 0.0) : zc(0.0, 0.0);
    }
    if (!any) break;
    DP_HIP(hipMemcpyAsync(scl, sbuf, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    scale_cols<<<g1(blk), 256, 0, st>>>(Rp, Vp, scl, n, nrhs);
    int kdone = 0;
    for (int k = 0; k < m; ++k) {
      cplx* vk = Vp + k * blk;
      cplx* zk = Zp + k * blk;
      if (pre) {
        ta.start(st);
        DP_TRY(precond_apply(p, nrhs, vk, zk, prec));
        ta.stop(st);
        ++applies;
      }
      tm.start(st);
      DP_TRY(matvec(p, nrhs, zk, Wp, prec));
      tm.stop(st);
      DP_HIP(hipEventRecord(ev_mv.e, st));
      ++matvecs;
      const int kp1 = k + 1;
      gram_dots<<<dim3(nbx, nrhs), 256, 0, st>>>(Vp, blk, Wp, n, nrhs, kp1, part.as<cplx>());
      gram_reduce<<<(kp1 * nrhs + 255) / 256, 256, 0, st>>>(part.as<cplx>(), nbx, kp1, nrhs, h1);
      if (kp1 <= kFuseK) {
        gram_update_dots<<<dim3(nbx, nrhs), 256, 0, st>>>(Vp, blk, Wp, h1, n, nrhs, kp1, part.as<cplx>());
      } else {
        gram_update<<<g1(blk), 256, 0, st>>>(Vp, blk, Wp, h1, n, nrhs, kp1);
        gram_dots<<<dim3(nbx, nrhs), 256, 0, st>>>(Vp, blk, Wp, n, nrhs, kp1, part.as<cplx>());
      }
      gram_reduce<<<(kp1 * nrhs + 255) / 256, 256, 0, st>>>(part.as<cplx>(), nbx, kp1, nrhs, h2);
      gram_update<<<g1(blk), 256, 0, st>>>(Vp, blk, Wp, h2, n, nrhs, kp1);
      {
        double* pp = reinterpret_cast<double*>(part.as<cplx>());
        col_norm2<<<dim3(nbx, nrhs), 256, 0, st>>>(Wp, n, nrhs, pp);
        norm_reduce<<<(nrhs + 63) / 64, 64, 0, st>>>(pp, nbx, nrhs, nrm);
      }
      // h1, h2 and the norms in one copy (h2 and the norms sit at fixed offsets)
      DP_HIP(hipMemcpyAsync(hbuf, h1, 2 * hsz * sizeof(cplx) + nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
      DP_HIP(hipEventRecord(ev_rb.e, st));
      // sleep through the matrix-vector product, then poll the readback
      // through the short orthogonalisation tail (a blocking wait there would
      // add the thread's wake-up to every step), yielding the core between
      // polls and blocking after 2 ms
      DP_TRY(wait_event(ev_mv.e, 0));
      DP_TRY(wait_event(ev_rb.e, 2000));
      tm.collect();
      ta.collect();
      p->clock.collect();
      p->clock32.collect();
      bool still = false;
      for (int c = 0; c < nrhs; ++c) {
        sbuf[c] = 0.0;
        if (!active[c]) continue;
        for (int i = 0; i <= k; ++i) {
          const cplx a = hbuf[(size_t)i * nrhs + c], b = hbuf[hsz + (size_t)i * nrhs + c];
          Hat(i, k, c) = zc(a.re + b.re, a.im + b.im);
        }
        const double hn = sqrt(nbuf[c]);
        Hat(k + 1, k, c) = zc(hn, 0.0);
        for (int i = 0; i < k; ++i) {  // Q_i = [[conj c, conj s], [-s, c]]
          const zc ci = cs[(size_t)c * m + i], si = sn[(size_t)c * m + i];
          const zc t = std::conj(ci) * Hat(i, k, c) + std::conj(si) * Hat(i + 1, k, c);
          Hat(i + 1, k, c) = -si * Hat(i, k, c) + ci * Hat(i + 1, k, c);
          Hat(i, k, c) = t;
        }
        const zc a = Hat(k, k, c), b = Hat(k + 1, k, c);
        const double den = sqrt(std::norm(a) + std::norm(b));
        const zc ck = den > 0 ? a / den : zc(1.0, 0.0), sk = den > 0 ? b / den : zc(0.0, 0.0);
        cs[(size_t)c * m + k] = ck;
        sn[(size_t)c * m + k] = sk;
        Hat(k, k, c) = den;
        Hat(k + 1, k, c) = 0.0;
        zc& gk = g[(size_t)c * (m + 1) + k];
        g[(size_t)c * (m + 1) + k + 1] = -sk * gk;
        gk = std::conj(ck) * gk;
        its[c] += 1;
        kc[c] = k + 1;
        const double est = std::abs(g[(size_t)c * (m + 1) + k + 1]) / fn[c];
        rel[c] = est;
        if (est <= tol || hn == 0.0 || its[c] >= o->max_iters) {
          active[c] = 0;
          conv_est[c] = est <= tol || hn == 0.0;
        } else {
          sbuf[c] = 1.0 / hn;
          still = true;
        }
      }
      kdone = k + 1;
      if (!still) break;
      DP_HIP(hipMemcpyAsync(scl, sbuf, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
      scale_cols<<<g1(blk), 256, 0, st>>>(Wp, Vp + (k + 1) * blk, scl, n, nrhs);
    }
    // y = H^{-1} g per column (upper triangular), X += Z y
    std::fill(yh.begin(), yh.end(), cplx{0.0, 0.0});
    for (int c = 0; c < nrhs; ++c) {
      const int kk = kc[c];
      std::vector<zc> y(kk);
      for (int i = kk - 1; i >= 0; --i) {
        zc s = g[(size_t)c * (m + 1) + i];
        for (int j = i + 1; j < kk; ++j) s -= Hat(i, j, c) * y[j];
        y[i] = s / Hat(i, i, c);
      }
      for (int i = 0; i < kk; ++i) yh[(size_t)i * nrhs + c] = {y[i].real(), y[i].imag()};
    }
    DP_HIP(hipMemcpyAsync(ydev, yh.data(), (size_t)kdone * nrhs * sizeof(cplx), hipMemcpyHostToDevice, st));
    combine<<<g1(blk), 256, 0, st>>>(Zp, blk, X, ydev, n, nrhs, kdone);
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
    tm.collect();
    p->clock.collect();
    p->clock32.collect();
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
  if (info) {
    info->iters_max = imax;
    info->matvecs = matvecs;
    info->applies = applies;
    info->relres_max = rmax;
    info->t_matvec = tm.acc;
    info->t_apply = ta.acc;
    info->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_krylov = info->t_total - tm.acc - ta.acc;
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
  DP_HIP(hipMemcpyAsync(R.p, F, blk * sizeof(cplx), hipMemcpyDeviceToDevice, st));
  std::vector<int64_t> its(nrhs, 0), its_in(nrhs);
  std::vector<double> rel(nrhs, 1.0), rel_in(nrhs), kv(nrhs);
  for (int c = 0; c < nrhs; ++c) rel[c] = fn[c] > 0 ? 1.0 : 0.0;
  dp_solve_opts oi = *o;
  oi.tol = o->inner_tol;
  int64_t mv = 0, mv32 = 0, ap = 0, outer = 0;
  double t_mv = 0, t_ap = 0;
  Timer tm;
  tm.init();
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
    info->t_matvec = t_mv + tm.acc;
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
