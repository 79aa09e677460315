// Per-problem device tables, plane-wave data and the Hankel test hook.
//
// Kress correction table (product quadrature for log(4 sin^2((t-tau)/2)),
// n = 2N nodes):
//   R_k = -(2 pi/N) sum_{m=1}^{N-1} cos(m k pi/N)/m - (pi/N^2) cos(k pi)
//   C_k = R_k - (2 pi/n) log(4 sin^2(pi k/n)),  k = 1..n-1;  C_0 := R_0.
// The sweep uses A_ij = (2 pi/n)|x'_j| K + C_{(i-j) mod n} |x'_j| K1 off the
// diagonal, which equals R_{|i-j|} K1 + (pi/N) K2 with K2 = K - K1 log(...)
// without forming the cancelling difference.  The cosine sums of R_k are the
// real part of the DFT of the sequence 1/m (m = 1..N-1): one FFT for
// power-of-two n, else a fixed-order block reduction per k.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dp_internal.hpp"

namespace dp {

// cos(2 pi l/n) and e^{-2 pi i l/n} tables, from sincospi of an exact ratio.
__global__ void trig_tables(double* ct, cplx* tw, int n) {
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n; l += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(2.0 * l / n, &s, &c);
    ct[l] = c;
    if (tw) tw[l] = {c, -s};
  }
}

// One block per k: R_k by a fixed-order block reduction; then C_k.
__global__ __launch_bounds__(256) void kress_table(const double* __restrict__ ct, double* C, int n) {
  const int k = blockIdx.x;
  const int N = n / 2;
  __shared__ double red[256];
  double acc = 0.0;
  long long l = ((long long)threadIdx.x * k) % n;  // (m k) mod n for m = threadIdx.x (+256 steps)
  const long long step = (256LL * k) % n;
  for (int m = threadIdx.x; m < N; m += 256) {
    if (m >= 1) acc += ct[l] / (double)m;
    l += step;
    if (l >= n) l -= n;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double R = -(2.0 * kPi / N) * red[0] - (kPi / ((double)N * N)) * ((k & 1) ? -1.0 : 1.0);
    if (k == 0) {
      C[0] = R;
    } else {
      const double sn = sinpi((double)k / n);
      C[k] = R - (2.0 * kPi / n) * log(4.0 * sn * sn);
    }
  }
}

// a_m = 1/m for 1 <= m < N, 0 otherwise (length n = 2N): Re DFT(a)_k is the
// sum in R_k.
__global__ void kress_seq(cplx* a, int n) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n; m += gridDim.x * blockDim.x)
    a[m] = {(m >= 1 && m < n / 2) ? 1.0 / m : 0.0, 0.0};
}

// R_k = -(2 pi/N) Re A_k - (pi/N^2) (-1)^k from A = DFT(a) as the FFT leaves
// it (n = n1 n2: A_k at position n2 (k mod n1) + k / n1); then C_k.
__global__ void kress_from_dft(const cplx* __restrict__ A, double* C, int n, int n1, int n2) {
  const int N = n / 2;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double Ak = A[(size_t)n2 * (k % n1) + k / n1].re;
    const double R = -(2.0 * kPi / N) * Ak - (kPi / ((double)N * N)) * ((k & 1) ? -1.0 : 1.0);
    if (k == 0) {
      C[0] = R;
    } else {
      const double sn = sinpi((double)k / n);
      C[k] = R - (2.0 * kPi / n) * log(4.0 * sn * sn);
    }
  }
}

int build_tables(dp_problem* p) {
  const int n = (int)p->n;
  hipStream_t st = p->ctx->stream;
  DevBuf ct;
  DP_TRY(ct.reserve(n * sizeof(double)));
  DP_TRY(p->C.reserve(n * sizeof(double)));
  cplx* tw = nullptr;
  if ((n & (n - 1)) == 0) {  // FFT twiddles for the spectral derivative (power-of-two n)
    DP_TRY(p->twiddle.reserve(n * sizeof(cplx)));
    tw = p->twiddle.as<cplx>();
  }
  trig_tables<<<(n + 255) / 256, 256, 0, st>>>(ct.as<double>(), tw, n);
  if (tw) {
    // power-of-two n: the sums of R_k as one FFT of the sequence 1/m
    DevBuf a;
    DP_TRY(a.reserve((size_t)n * sizeof(cplx)));
    kress_seq<<<(n + 255) / 256, 256, 0, st>>>(a.as<cplx>(), n);
    int n1 = 0, n2 = 0;
    fft_inplace(p, a.as<cplx>(), 1, -1, &n1, &n2);
    kress_from_dft<<<(n + 255) / 256, 256, 0, st>>>(a.as<cplx>(), p->C.as<double>(), n, n1, n2);
    DP_HIP(hipGetLastError());
    a.release();
  } else {
    kress_table<<<n, 256, 0, st>>>(ct.as<double>(), p->C.as<double>(), n);
  }
  DP_HIP(hipGetLastError());
  std::vector<double> hc(n);
  DP_HIP(hipMemcpyAsync(hc.data(), p->C.as<double>(), n * sizeof(double), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  p->R0 = hc[0];
  p->cmax = 0;
  for (int k = 1; k < n; ++k) p->cmax = std::max(p->cmax, std::fabs(hc[k]));
  // FP32 copy for the single-precision sweep, as the ratio C_k / (pi dt) of
  // the Kress weight to the trapezoid weight (both times |x'_j|/4)
  std::vector<float> hc32(n);
  for (int k = 0; k < n; ++k) hc32[k] = (float)(hc[k] * (double)n / (2.0 * kPi * kPi));
  DP_TRY(p->C32.reserve(n * sizeof(float)));
  DP_HIP(hipMemcpyAsync(p->C32.p, hc32.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
  DP_HIP(hipStreamSynchronize(st));
  ct.release();
  return DP_OK;
}

// f = -exp(i omega d.x) (soft) or -i omega (d.nu) exp(i omega d.x) (hard)
__global__ void plane_wave(const SrcRec* __restrict__ src, const double* __restrict__ ang, cplx* f, int n,
                           int nrhs, double omega, int kind) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = idx % n;
    const int c = idx / n;
    double dy, dx;
    dp_sincos(ang[c], dy, dx);
    const SrcRec s = src[i];
    double sn, cs;
    dp_sincos(omega * (dx * s.x + dy * s.y), sn, cs);
    if (kind == DP_SOFT) {
      f[idx] = {-cs, -sn};
    } else {
      const double a = omega * (dx * s.nx + dy * s.ny);
      // -i a (cs + i sn) = a sn - i a cs
      f[idx] = {a * sn, -a * cs};
    }
  }
}

int rhs_plane_wave(dp_problem* p, int nrhs, const double* angles_dev, cplx* f) {
  const size_t tot = (size_t)p->n * nrhs;
  size_t g = (tot + 255) / 256;
  plane_wave<<<(int)(g > 8192 ? 8192 : g), 256, 0, p->ctx->stream>>>(p->src.as<SrcRec>(), angles_dev, f,
                                                                       (int)p->n, nrhs, p->omega, p->kind);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

__global__ void hankel_kernel(const double* __restrict__ z, double* out, int64_t m) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const H01 h = hankel01(z[k]);
    out[4 * k + 0] = h.h0.re;
    out[4 * k + 1] = h.h0.im;
    out[4 * k + 2] = h.h1.re;
    out[4 * k + 3] = h.h1.im;
  }
}

int hankel_eval_dev(int64_t m, const double* z, double* out, hipStream_t s) {
  int64_t g = (m + 255) / 256;
  hankel_kernel<<<(int)(g > 4096 ? 4096 : (g ? g : 1)), 256, 0, s>>>(z, out, m);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

}  // namespace dp
