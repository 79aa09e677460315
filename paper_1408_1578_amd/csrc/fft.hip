// Arclength derivative of the trigonometric interpolant (Nyquist mode
// dropped), used by Maue's form of the hypersingular operator:
//   (D_s phi)_i = (1/|x'(t_i)|) * IDFT( i m DFT(phi) )_i,  m in (-n/2, n/2).
// Radix-2 FFT for power-of-two lengths, batched over columns; any other even
// n goes through Bluestein's chirp-z identity (below).  Length <= 4096: one
// line per column, transformed in LDS.  Larger n: four-step with
// n = n1 * n2 (n1, n2 <= 4096): length-n1 transforms over the stride-n2
// index with the twiddle e^{-+2 pi i j2 k1/n}, then length-n2 transforms of
// contiguous lines; the spectrum is left in the transposed order
// X[k1 + n1 k2] at position n2 k1 + k2, multiplied there, and the inverse
// runs the two passes in reverse order.
#include "dp_internal.hpp"

namespace dp {

constexpr int kFftLds = 4096;  // complex elements per block
// threads per block of the LDS passes, and elements per block of the
// column and row passes (at n = 32768 x 64 columns: 106 us per derivative
// against 116 with 256 threads and 4096-element blocks; Bluestein's
// length-65536 transforms for n = 24576: 427 us per derivative against 447;
// more blocks in flight per CU hide more of the load latency)
constexpr int kFftThreads = 512;
constexpr int kFftTile = 2048;

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) { return __brev(v) >> (32 - bits); }

// In-LDS DIT transform of `lines` lines of length Lf stored as
// buf[e * lines + l] (element-major, so that loads over lines coalesce).
// Input must be in bit-reversed element order.  dir = -1 forward, +1 inverse.
// Lf, lines and ntw are powers of two (loglines = log2 lines).  The radix-2
// stages of half sizes h and 2h are done together as one radix-4 stage
// (elements pos, pos + h, pos + 2h, pos + 3h of a block of 4h: twiddles
// W_2h^pos for the first pair of butterflies, W_4h^pos and
// W_4h^(pos + h) = W_4h^pos (-+i) for the second); one plain radix-2 stage
// comes first when log2 Lf is odd.  Half the stages, barriers and LDS round
// trips of the radix-2 form, with the same pairing and output order.
__device__ void lds_fft(cplx* buf, int Lf, int lines, int loglines, const cplx* tw, int ntw, int dir) {
  int half = 1;
  if (__builtin_ctz(Lf) & 1) {  // half = 1: the twiddle is 1
    const int nb = (Lf >> 1) * lines;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
      const int l = t & (lines - 1);
      const int i0 = (t >> loglines) << 1;
      const cplx a = buf[i0 * lines + l], c = buf[(i0 + 1) * lines + l];
      buf[i0 * lines + l] = {a.re + c.re, a.im + c.im};
      buf[(i0 + 1) * lines + l] = {a.re - c.re, a.im - c.im};
    }
    __syncthreads();
    half = 2;
  }
  for (; half < Lf; half <<= 2) {
    const int h = half;
    const int nb = (Lf >> 2) * lines;
    const int s1 = ntw / (2 * h), s2 = ntw / (4 * h);
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
      const int l = t & (lines - 1);
      const int b = t >> loglines;  // radix-4 butterfly, [0, Lf / 4)
      const int pos = b & (h - 1);
      const int i0 = ((b - pos) << 2) + pos;
      cplx w1 = tw[pos * s1], w2 = tw[pos * s2];
      if (dir > 0) {
        w1.im = -w1.im;
        w2.im = -w2.im;
      }
      cplx* p0 = buf + (size_t)i0 * lines + l;
      const size_t hs = (size_t)h * lines;
      const cplx a0 = p0[0], a1 = p0[hs], a2 = p0[2 * hs], a3 = p0[3 * hs];
      const cplx m1 = cmul(a1, w1), m3 = cmul(a3, w1);
      const cplx t0 = {a0.re + m1.re, a0.im + m1.im}, t1 = {a0.re - m1.re, a0.im - m1.im};
      const cplx t2 = {a2.re + m3.re, a2.im + m3.im}, t3 = {a2.re - m3.re, a2.im - m3.im};
      const cplx u2 = cmul(t2, w2), u3 = cmul(t3, w2);
      const cplx v3 = dir < 0 ? cplx{u3.im, -u3.re} : cplx{-u3.im, u3.re};  // W_4h^h = -i (forward), +i
      p0[0] = {t0.re + u2.re, t0.im + u2.im};
      p0[2 * hs] = {t0.re - u2.re, t0.im - u2.im};
      p0[hs] = {t1.re + v3.re, t1.im + v3.im};
      p0[3 * hs] = {t1.re - v3.re, t1.im - v3.im};
    }
    __syncthreads();
  }
}

// Column pass: for each column b and each j2 in [0, n2): line over j1 (stride
// n2).  Optional twiddle e^{dir 2 pi i j2 k1/n}: applied after the transform
// (forward) or before it (inverse).
// `in` may equal `data` (in place: a block reads all its lines before it
// writes).  With `speed`, each written element is divided by the speed of
// its node (the last pass of the inverse transform is in natural order).
__global__ __launch_bounds__(kFftThreads) void fft_col_pass(const cplx* in, cplx* data, int n, int n1, int n2, int logn1, int lines,
                             const cplx* __restrict__ tw, int dir, int twiddle, const SrcRec* __restrict__ speed) {
  extern __shared__ cplx sbuf[];
  const int b = blockIdx.y;
  const int j2_0 = blockIdx.x * lines;
  const int loglines = __builtin_ctz(lines);
  cplx* base = data + (size_t)b * n;
  const cplx* ibase = in + (size_t)b * n;
  for (int t = threadIdx.x; t < n1 * lines; t += blockDim.x) {
    const int l = t & (lines - 1), j1 = t >> loglines;
    cplx v = ibase[(size_t)n2 * j1 + j2_0 + l];
    if (twiddle && dir > 0) {  // inverse: pre-twiddle e^{+2 pi i j2 k1/n} (k1 = j1 here)
      cplx w = tw[((j2_0 + l) * j1) & (n - 1)];
      w.im = -w.im;
      v = cmul(v, w);
    }
    sbuf[bitrev(j1, logn1) * lines + l] = v;
  }
  __syncthreads();
  lds_fft(sbuf, n1, lines, loglines, tw, n, dir);
  for (int t = threadIdx.x; t < n1 * lines; t += blockDim.x) {
    const int l = t & (lines - 1), k1 = t >> loglines;
    cplx v = sbuf[k1 * lines + l];
    if (twiddle && dir < 0) v = cmul(v, tw[((j2_0 + l) * k1) & (n - 1)]);
    const size_t o = (size_t)n2 * k1 + j2_0 + l;
    if (speed) {
      const double r = 1.0 / speed[o].sp;
      v = {v.re * r, v.im * r};
    }
    base[o] = v;
  }
}

// Row pass: lines of n2 contiguous elements starting at n2 * k1.
__global__ __launch_bounds__(kFftThreads) void fft_row_pass(cplx* data, int n, int n2, int logn2, int lines, const cplx* __restrict__ tw,
                             int dir) {
  extern __shared__ cplx sbuf[];
  const int b = blockIdx.y;
  const int k1_0 = blockIdx.x * lines;
  cplx* base = data + (size_t)b * n + (size_t)k1_0 * n2;
  for (int t = threadIdx.x; t < n2 * lines; t += blockDim.x) {
    const int e = t & (n2 - 1), l = t >> logn2;
    sbuf[bitrev(e, logn2) * lines + l] = base[(size_t)l * n2 + e];
  }
  __syncthreads();
  lds_fft(sbuf, n2, lines, __builtin_ctz(lines), tw, n, dir);
  for (int t = threadIdx.x; t < n2 * lines; t += blockDim.x) {
    const int e = t & (n2 - 1), l = t >> logn2;
    base[(size_t)l * n2 + e] = sbuf[e * lines + l];
  }
}

// Row pass of the derivative: per line (fixed k1) the forward transform over
// j2, the multiplication of X[k1 + n1 k2] by i m / n (m the signed
// frequency, Nyquist zeroed), and the inverse transform back over j2, all in
// LDS.
__global__ __launch_bounds__(kFftThreads) void fft_row_deriv(cplx* data, int n, int n1, int n2, int logn2, int lines, const cplx* __restrict__ tw) {
  extern __shared__ cplx sbuf[];
  const int b = blockIdx.y;
  const int k1_0 = blockIdx.x * lines;
  const int loglines = __builtin_ctz(lines);
  cplx* base = data + (size_t)b * n + (size_t)k1_0 * n2;
  for (int t = threadIdx.x; t < n2 * lines; t += blockDim.x) {
    const int e = t & (n2 - 1), l = t >> logn2;
    sbuf[bitrev(e, logn2) * lines + l] = base[(size_t)l * n2 + e];
  }
  __syncthreads();
  lds_fft(sbuf, n2, lines, loglines, tw, n, -1);
  // scale, then put the spectrum into bit-reversed order for the inverse:
  // every element is read (into registers) before any is overwritten
  constexpr int PER = kFftLds / kFftThreads;  // blockDim.x == kFftThreads, n2 * lines <= kFftLds
  cplx tmp[PER];
  int dst[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = threadIdx.x + kFftThreads * q;
    dst[q] = -1;
    if (t < n2 * lines) {
      const int e = t & (n2 - 1), l = t >> logn2;
      const int k = k1_0 + l + n1 * e;
      const int m = (k < n / 2) ? k : ((k == n / 2) ? 0 : k - n);
      const double fm = (double)m / n;
      const cplx v = sbuf[e * lines + l];
      tmp[q] = {-fm * v.im, fm * v.re};
      dst[q] = bitrev(e, logn2) * lines + l;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q)
    if (dst[q] >= 0) sbuf[dst[q]] = tmp[q];
  __syncthreads();
  lds_fft(sbuf, n2, lines, loglines, tw, n, +1);
  for (int t = threadIdx.x; t < n2 * lines; t += blockDim.x) {
    const int e = t & (n2 - 1), l = t >> logn2;
    base[(size_t)l * n2 + e] = sbuf[e * lines + l];
  }
}

// Spectrum at position p = n2 k1 + k2 holds X[k1 + n1 k2]: multiply by
// i m / n (m the signed frequency, Nyquist zeroed).
__global__ void deriv_scale(cplx* data, int n, int n1, int n2, int nb) {
  const size_t tot = (size_t)n * nb;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(idx & (size_t)(n - 1));  // n, n2 powers of two
    const int k1 = p / n2, k2 = p & (n2 - 1);
    const int k = k1 + n1 * k2;
    const int m = (k < n / 2) ? k : ((k == n / 2) ? 0 : k - n);
    const cplx v = data[idx];
    const double f = (double)m / n;
    data[idx] = {-f * v.im, f * v.re};
  }
}

__global__ void copy_div_speed(const cplx* __restrict__ in, cplx* __restrict__ out, const SrcRec* __restrict__ src,
                               int n, size_t tot, int divide) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    cplx v = in[idx];
    if (divide) {
      const double s = 1.0 / src[idx & (size_t)(n - 1)].sp;  // n a power of two
      v = {v.re * s, v.im * s};
    }
    out[idx] = v;
  }
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// In-place transform of nb contiguous columns of length N (a power of two,
// at most 2^24) with the twiddle table tw[l] = e^{-2 pi i l/N}: dir = -1
// forward, +1 inverse (unnormalised).
static void fft_run(cplx* d, int N, const cplx* tw, int nb, int dir, hipStream_t st) {
  const int logn = ilog2(N);
  const int log1 = logn <= 12 ? logn : (logn + 1) / 2;
  const int log2n = logn - log1;
  const int n1 = 1 << log1, n2 = 1 << log2n;
  auto col = [&](int dirc) {
    int lines = kFftTile / n1;
    if (lines > n2) lines = n2;
    if (lines < 1) lines = 1;
    dim3 g(n2 / lines, nb);
    fft_col_pass<<<g, kFftThreads, (size_t)n1 * lines * sizeof(cplx), st>>>(d, d, N, n1, n2, log1, lines, tw, dirc,
                                                                     n2 > 1, nullptr);
  };
  auto row = [&](int dirc) {
    if (n2 == 1) return;
    int lines = kFftTile / n2;
    if (lines > n1) lines = n1;
    if (lines < 1) lines = 1;
    dim3 g(n1 / lines, nb);
    fft_row_pass<<<g, kFftThreads, (size_t)n2 * lines * sizeof(cplx), st>>>(d, N, n2, log2n, lines, tw, dirc);
  };
  if (dir < 0) {
    col(-1);
    row(-1);
  } else {
    row(+1);
    col(+1);
  }
}

static void fft_passes(dp_problem* p, cplx* d, int nb, int dir) {
  fft_run(d, (int)p->n, p->twiddle.as<cplx>(), nb, dir, p->ctx->stream);
}

void fft_inplace(dp_problem* p, cplx* d, int nb, int dir, int* n1, int* n2) {
  const int logn = ilog2((int)p->n);
  const int log1 = logn <= 12 ? logn : (logn + 1) / 2;
  *n1 = 1 << log1;
  *n2 = 1 << (logn - log1);
  fft_passes(p, d, nb, dir);
}

static int grid_for(size_t tot) {
  const size_t g = (tot + 255) / 256;
  return (int)(g > 8192 ? 8192 : g);
}

// ------------------------------------------------------------------ Bluestein
// For n not a power of two the length-n DFT X_k = sum_j phi_j e^{-2 pi i jk/n}
// follows from jk = (j^2 + k^2 - (k - j)^2)/2 as a convolution:
//   X_k = conj(c_k) sum_j (phi_j conj(c_j)) c_{k-j},   c_j = e^{i pi j^2/n},
// evaluated by power-of-two FFTs of length M >= 2n - 1 of the zero-padded
// sequence and of b (c_l at l and M - l, l < n).  The inverse DFT is the
// same with the chirp conjugated: u_j = c_j sum_k (U_k c_k) conj(c)_{j-k};
// as b is symmetric (b_l = b_{M-l}), FFT_M(conj b) = conj(FFT_M(b)).  The
// chirp phase is reduced exactly, pi (j^2 mod 2n)/n, before sincospi.

__global__ void blu_tables(cplx* chirp, cplx* b, cplx* tw, int n, int M) {
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < M; l += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(2.0 * l / M, &s, &c);
    tw[l] = {c, -s};
    const int j = l < n ? l : (l > M - n ? M - l : -1);
    cplx v = {0.0, 0.0};
    if (j >= 0) {
      const long long r = ((long long)j * j) % (2LL * n);
      sincospi((double)r / n, &s, &c);
      v = {c, s};
      if (l < n) chirp[l] = v;
    }
    b[l] = v;
  }
}

// a[col][j] = in[col][j] conj(c_j) (j < n), 0 up to M
__global__ void blu_premul(const cplx* __restrict__ in, cplx* __restrict__ a, const cplx* __restrict__ chirp,
                           int n, int M, int nb) {
  const size_t tot = (size_t)M * nb;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % (size_t)M);
    const size_t col = idx / (size_t)M;
    cplx v = {0.0, 0.0};
    if (j < n) {
      const cplx x = in[col * n + j], c = chirp[j];
      v = {x.re * c.re + x.im * c.im, x.im * c.re - x.re * c.im};
    }
    a[idx] = v;
  }
}

// a *= B (or conj B) / M
__global__ void blu_mul(cplx* a, const cplx* __restrict__ B, int M, int nb, int conjB) {
  const size_t tot = (size_t)M * nb;
  const double s = 1.0 / M;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    cplx w = B[idx % (size_t)M];
    if (conjB) w.im = -w.im;
    const cplx v = cmul(a[idx], w);
    a[idx] = {v.re * s, v.im * s};
  }
}

// Between the two convolutions: X_k = conj(c_k) a_k; U_k = i m_k X_k / n
// (m_k the signed frequency, Nyquist zeroed); a_k = U_k c_k (k < n), 0 up to M.
__global__ void blu_mid(cplx* a, const cplx* __restrict__ chirp, int n, int M, int nb) {
  const size_t tot = (size_t)M * nb;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx % (size_t)M);
    cplx v = {0.0, 0.0};
    if (k < n) {
      const cplx c = chirp[k], y = a[idx];
      const cplx X = {y.re * c.re + y.im * c.im, y.im * c.re - y.re * c.im};
      const int m = (k < n / 2) ? k : ((k == n / 2) ? 0 : k - n);
      const double f = (double)m / n;
      const cplx U = {-f * X.im, f * X.re};
      v = cmul(U, c);
    }
    a[idx] = v;
  }
}

// out[col][j] = c_j a[col][j] (divided by the speed of node j with `src`)
__global__ void blu_post(const cplx* __restrict__ a, cplx* __restrict__ out, const cplx* __restrict__ chirp,
                         const SrcRec* __restrict__ src, int n, int M, int nb) {
  const size_t tot = (size_t)n * nb;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % (size_t)n);
    const size_t col = idx / (size_t)n;
    cplx v = cmul(chirp[j], a[col * M + j]);
    if (src) {
      const double r = 1.0 / src[j].sp;
      v = {v.re * r, v.im * r};
    }
    out[idx] = v;
  }
}

// Fused passes of a Bluestein derivative when M = n1 n2 takes the four-step
// path (n2 > 1): five passes instead of the thirteen of the separate
// transforms and pointwise kernels, with the same operations in the same
// order.  Column pass modes (each block: `lines` lines j2 over j1):
//   kBluPre : a = forward column transform of in conj(c) (zero for j >= n);
//   kBluMid : inverse column transform, the step between the convolutions
//             (blu_mid), forward column transform, in place on a;
//   kBluPost: inverse column transform, out = c a (divided by the speed
//             with src), j < n.
enum { kBluPre = 0, kBluMid = 1, kBluPost = 2 };
template <int MODE>
__global__ __launch_bounds__(kFftThreads) void blu_col(const cplx* __restrict__ in, cplx* a, cplx* __restrict__ out,
                                                       const cplx* __restrict__ chirp, const SrcRec* __restrict__ src,
                                                       int n, int M, int n1, int n2, int logn1, int lines,
                                                       const cplx* __restrict__ tw) {
  extern __shared__ cplx sbuf[];
  const size_t b = blockIdx.y;
  const int j2_0 = blockIdx.x * lines;
  const int loglines = __builtin_ctz(lines);
  cplx* ab = a + b * M;
  for (int t = threadIdx.x; t < n1 * lines; t += blockDim.x) {
    const int l = t & (lines - 1), j1 = t >> loglines;
    const int j = n2 * j1 + j2_0 + l;
    cplx v;
    if (MODE == kBluPre) {
      v = {0.0, 0.0};
      if (j < n) {
        const cplx x = in[b * n + j], c = chirp[j];
        v = {x.re * c.re + x.im * c.im, x.im * c.re - x.re * c.im};
      }
    } else {  // inverse: pre-twiddle e^{+2 pi i j2 k1/M} (k1 = j1 here)
      v = ab[j];
      cplx w = tw[((j2_0 + l) * j1) & (M - 1)];
      w.im = -w.im;
      v = cmul(v, w);
    }
    sbuf[bitrev(j1, logn1) * lines + l] = v;
  }
  __syncthreads();
  if (MODE != kBluPre) {
    lds_fft(sbuf, n1, lines, loglines, tw, M, +1);
    if (MODE == kBluMid) {
      // natural index k = n2 k1 + j2 at sbuf[k1 lines + l]: the step between
      // the convolutions, then into bit-reversed order for the forward
      // transform (every element read before any is overwritten)
      constexpr int PER = kFftLds / kFftThreads;
      cplx tmp[PER];
      int dst[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int t = threadIdx.x + kFftThreads * q;
        dst[q] = -1;
        if (t < n1 * lines) {
          const int l = t & (lines - 1), k1 = t >> loglines;
          const int k = n2 * k1 + j2_0 + l;
          cplx v = {0.0, 0.0};
          if (k < n) {
            const cplx c = chirp[k], y = sbuf[k1 * lines + l];
            const cplx X = {y.re * c.re + y.im * c.im, y.im * c.re - y.re * c.im};
            const int m = (k < n / 2) ? k : ((k == n / 2) ? 0 : k - n);
            const double f = (double)m / n;
            const cplx U = {-f * X.im, f * X.re};
            v = cmul(U, c);
          }
          tmp[q] = v;
          dst[q] = bitrev(k1, logn1) * lines + l;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (dst[q] >= 0) sbuf[dst[q]] = tmp[q];
      __syncthreads();
    }
  }
  if (MODE != kBluPost) lds_fft(sbuf, n1, lines, loglines, tw, M, -1);
  for (int t = threadIdx.x; t < n1 * lines; t += blockDim.x) {
    const int l = t & (lines - 1), k1 = t >> loglines;
    const int o = n2 * k1 + j2_0 + l;
    cplx v = sbuf[k1 * lines + l];
    if (MODE == kBluPost) {
      if (o < n) {
        v = cmul(chirp[o], v);
        if (src) {
          const double r = 1.0 / src[o].sp;
          v = {v.re * r, v.im * r};
        }
        out[b * n + o] = v;
      }
    } else {  // forward: post-twiddle e^{-2 pi i j2 k1/M}
      v = cmul(v, tw[((j2_0 + l) * k1) & (M - 1)]);
      ab[o] = v;
    }
  }
}

// Row pass of a Bluestein convolution: per line (fixed k1) the forward
// transform over k2, a *= B (conj B with conjB) / M at the spectrum
// positions n2 k1 + k2 (the layout B itself has), and the inverse transform.
__global__ __launch_bounds__(kFftThreads) void blu_row_conv(cplx* a, int M, int n2, int logn2, int lines,
                                                            const cplx* __restrict__ tw, const cplx* __restrict__ B,
                                                            int conjB) {
  extern __shared__ cplx sbuf[];
  const size_t b = blockIdx.y;
  const int k1_0 = blockIdx.x * lines;
  const int loglines = __builtin_ctz(lines);
  cplx* base = a + b * M + (size_t)k1_0 * n2;
  const cplx* Bb = B + (size_t)k1_0 * n2;
  for (int t = threadIdx.x; t < n2 * lines; t += blockDim.x) {
    const int e = t & (n2 - 1), l = t >> logn2;
    sbuf[bitrev(e, logn2) * lines + l] = base[(size_t)l * n2 + e];
  }
  __syncthreads();
  lds_fft(sbuf, n2, lines, loglines, tw, M, -1);
  constexpr int PER = kFftLds / kFftThreads;  // n2 * lines <= kFftLds
  const double s = 1.0 / M;
  cplx tmp[PER];
  int dst[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = threadIdx.x + kFftThreads * q;
    dst[q] = -1;
    if (t < n2 * lines) {
      const int e = t & (n2 - 1), l = t >> logn2;
      cplx w = Bb[(size_t)l * n2 + e];
      if (conjB) w.im = -w.im;
      const cplx v = cmul(sbuf[e * lines + l], w);
      tmp[q] = {v.re * s, v.im * s};
      dst[q] = bitrev(e, logn2) * lines + l;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q)
    if (dst[q] >= 0) sbuf[dst[q]] = tmp[q];
  __syncthreads();
  lds_fft(sbuf, n2, lines, loglines, tw, M, +1);
  for (int t = threadIdx.x; t < n2 * lines; t += blockDim.x) {
    const int e = t & (n2 - 1), l = t >> logn2;
    base[(size_t)l * n2 + e] = sbuf[e * lines + l];
  }
}

int bluestein_init(dp_problem* p) {
  const int n = (int)p->n;
  int M = 1;
  while (M < 2 * n - 1) M <<= 1;
  p->blu_M = M;
  hipStream_t st = p->ctx->stream;
  DP_TRY(p->blu_tw.reserve((size_t)M * sizeof(cplx)));
  DP_TRY(p->blu_chirp.reserve((size_t)n * sizeof(cplx)));
  DP_TRY(p->blu_B.reserve((size_t)M * sizeof(cplx)));
  blu_tables<<<(M + 255) / 256, 256, 0, st>>>(p->blu_chirp.as<cplx>(), p->blu_B.as<cplx>(), p->blu_tw.as<cplx>(), n,
                                             M);
  fft_run(p->blu_B.as<cplx>(), M, p->blu_tw.as<cplx>(), 1, -1, st);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// out = d/dt in (trigonometric interpolant), or d/ds with `divide` (speed),
// for nb columns by Bluestein; in may equal out.
static int bluestein_derivative(dp_problem* p, const cplx* in, cplx* out, int nb, bool divide) {
  const int n = (int)p->n, M = p->blu_M;
  hipStream_t st = p->ctx->stream;
  DP_TRY(p->blu_ws.reserve((size_t)M * nb * sizeof(cplx)));
  cplx* a = p->blu_ws.as<cplx>();
  const cplx* c = p->blu_chirp.as<cplx>();
  const cplx* B = p->blu_B.as<cplx>();
  const cplx* tw = p->blu_tw.as<cplx>();
  const SrcRec* sp = divide ? p->src.as<SrcRec>() : nullptr;
  const int logM = ilog2(M);
  const int log1 = logM <= 12 ? logM : (logM + 1) / 2;
  const int n1 = 1 << log1, n2 = 1 << (logM - log1);
  if (n2 > 1) {  // four-step transforms: the fused passes
    int lc = kFftTile / n1;
    if (lc > n2) lc = n2;
    if (lc < 1) lc = 1;
    int lr = kFftTile / n2;
    if (lr > n1) lr = n1;
    if (lr < 1) lr = 1;
    const dim3 gc(n2 / lc, nb), gr(n1 / lr, nb);
    const size_t ldc = (size_t)n1 * lc * sizeof(cplx), ldr = (size_t)n2 * lr * sizeof(cplx);
    blu_col<kBluPre><<<gc, kFftThreads, ldc, st>>>(in, a, nullptr, c, nullptr, n, M, n1, n2, log1, lc, tw);
    blu_row_conv<<<gr, kFftThreads, ldr, st>>>(a, M, n2, logM - log1, lr, tw, B, 0);
    blu_col<kBluMid><<<gc, kFftThreads, ldc, st>>>(nullptr, a, nullptr, c, nullptr, n, M, n1, n2, log1, lc, tw);
    blu_row_conv<<<gr, kFftThreads, ldr, st>>>(a, M, n2, logM - log1, lr, tw, B, 1);
    blu_col<kBluPost><<<gc, kFftThreads, ldc, st>>>(nullptr, a, out, c, sp, n, M, n1, n2, log1, lc, tw);
    DP_HIP(hipGetLastError());
    return DP_OK;
  }
  const int gM = grid_for((size_t)M * nb);
  blu_premul<<<gM, 256, 0, st>>>(in, a, c, n, M, nb);
  fft_run(a, M, tw, nb, -1, st);
  blu_mul<<<gM, 256, 0, st>>>(a, B, M, nb, 0);
  fft_run(a, M, tw, nb, +1, st);
  blu_mid<<<gM, 256, 0, st>>>(a, c, n, M, nb);
  fft_run(a, M, tw, nb, -1, st);
  blu_mul<<<gM, 256, 0, st>>>(a, B, M, nb, 1);
  fft_run(a, M, tw, nb, +1, st);
  blu_post<<<grid_for((size_t)n * nb), 256, 0, st>>>(a, out, c, sp, n, M, nb);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// In place: d <- d/dt of each of nb columns (trigonometric interpolant).
static void t_derivative(dp_problem* p, cplx* d, int nb) {
  const int n = (int)p->n;
  fft_passes(p, d, nb, -1);
  const int logn = ilog2(n);
  const int log1 = logn <= 12 ? logn : (logn + 1) / 2;
  deriv_scale<<<grid_for((size_t)n * nb), 256, 0, p->ctx->stream>>>(d, n, 1 << log1, 1 << (logn - log1), nb);
  fft_passes(p, d, nb, +1);
}

int spectral_derivative(dp_problem* p, int nrhs, const cplx* in, cplx* out) {
  if (p->blu_M) return bluestein_derivative(p, in, out, nrhs, true);
  const int n = (int)p->n;
  const size_t tot = (size_t)n * nrhs;
  hipStream_t st = p->ctx->stream;
  const int logn = ilog2(n);
  const int log1 = logn <= 12 ? logn : (logn + 1) / 2;
  const int n1 = 1 << log1, n2 = 1 << (logn - log1);
  if (n2 > 1) {
    // four-step: forward column pass (reading `in`), fused row pass
    // (forward, derivative factor, inverse), inverse column pass dividing
    // by the speed
    const cplx* tw = p->twiddle.as<cplx>();
    int lc = kFftTile / n1;
    if (lc > n2) lc = n2;
    if (lc < 1) lc = 1;
    int lr = kFftTile / n2;
    if (lr > n1) lr = n1;
    if (lr < 1) lr = 1;
    const dim3 gc(n2 / lc, nrhs), gr(n1 / lr, nrhs);
    fft_col_pass<<<gc, kFftThreads, (size_t)n1 * lc * sizeof(cplx), st>>>(in, out, n, n1, n2, log1, lc, tw, -1, 1, nullptr);
    fft_row_deriv<<<gr, kFftThreads, (size_t)n2 * lr * sizeof(cplx), st>>>(out, n, n1, n2, logn - log1, lr, tw);
    fft_col_pass<<<gc, kFftThreads, (size_t)n1 * lc * sizeof(cplx), st>>>(out, out, n, n1, n2, log1, lc, tw, +1, 1,
                                                                  p->src.as<SrcRec>());
    DP_HIP(hipGetLastError());
    return DP_OK;
  }
  const int grid = grid_for(tot);
  copy_div_speed<<<grid, 256, 0, st>>>(in, out, p->src.as<SrcRec>(), n, tot, 0);
  t_derivative(p, out, nrhs);
  copy_div_speed<<<grid, 256, 0, st>>>(out, out, p->src.as<SrcRec>(), n, tot, 1);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// z[i] = x_i + i y_i, duplicated into the second column.
__global__ void pack_position(const SrcRec* __restrict__ src, cplx* z, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const cplx v = {src[i].x, src[i].y};
    z[i] = v;
    z[n + i] = v;
  }
}

// Column 0 holds z', column 1 holds z''.  Signed curvature of a
// counter-clockwise curve: (x' y'' - y' x'') / |z'|^3.
__global__ void curvature_from_derivs(const cplx* __restrict__ z, SrcRec* src, double* kap, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const cplx a = z[i], b = z[n + i];
    const double s2 = a.re * a.re + a.im * a.im;
    const double k = (a.re * b.im - a.im * b.re) / (s2 * sqrt(s2));
    src[i].kappa = k;
    kap[i] = k;
  }
}

int curvature_spectral(dp_problem* p, double* hkap) {
  const int n = (int)p->n;
  hipStream_t st = p->ctx->stream;
  DevBuf z;
  struct Release {
    DevBuf& b;
    ~Release() { b.release(); }
  } release{z};
  DP_TRY(z.reserve((size_t)2 * n * sizeof(cplx) + (size_t)n * sizeof(double)));
  cplx* zc = z.as<cplx>();
  double* kap = reinterpret_cast<double*>(zc + 2 * (size_t)n);
  const int grid = grid_for((size_t)n);
  pack_position<<<grid, 256, 0, st>>>(p->src.as<SrcRec>(), zc, n);
  if (p->blu_M) {
    DP_TRY(bluestein_derivative(p, zc, zc, 2, false));       // both columns: z'
    DP_TRY(bluestein_derivative(p, zc + n, zc + n, 1, false));  // second column: z''
  } else {
    t_derivative(p, zc, 2);   // both columns: z'
    t_derivative(p, zc + n, 1);  // second column: z''
  }
  curvature_from_derivs<<<grid, 256, 0, st>>>(zc, p->src.as<SrcRec>(), kap, n);
  DP_HIP(hipGetLastError());
  DP_HIP(hipMemcpyAsync(hkap, kap, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  return DP_OK;
}

}  // namespace dp
