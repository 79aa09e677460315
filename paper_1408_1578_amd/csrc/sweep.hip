// On-the-fly Nystrom matvec: every ordered pair (i, j) of boundary nodes is
// visited once per call; the Hankel kernels are evaluated in registers and
// never stored.
//
// Operators (Sec. 1) with G = (i/4) H0(omega r), r = |x_i - x_j|,
// rhat = (x_i - x_j)/r, trapezoid weight dt |x'_j| (dt = 2 pi/n) and the
// Kress correction C_{(i-j) mod n} |x'_j| K1 for the log-singular part K1:
//   S : K = (i/4) H0,                     K1 = -J0/(4 pi)
//   D : K = (i omega/4) H1 nu_j.rhat,     K1 = -(omega/(4 pi)) J1 nu_j.rhat
//   D': K = -(i omega/4) H1 nu_i.rhat,    K1 = (omega/(4 pi)) J1 nu_i.rhat
// A_ij = dt |x'_j| K + C_{i-j} |x'_j| K1 for i != j; the diagonal (Kress
// limits) is added in the epilogue.
//   soft (eq. (3)):   A = 1/2 I + D - i eta S                  (1 density)
//   hard (eq. (2)), Maue's identity N = D_s S D_s + omega^2 nu.S nu:
//     u = S (D_s q),  v = [-i (omega^2/eta)(nu_i.nu_j) S - D'] q   (2 densities)
//     A q = 1/2 q + v + (1/(i eta)) D_s u
//
// Launch shapes (gfx950, wave64):
//   private: nrp <= 4 columns.  256 threads = 256 target rows per block, one
//            row per lane; every wave evaluates its own kernel values and
//            multiplies them into nrp columns.  Source data is wave-uniform
//            (scalar loads).
//   shared : nrp = 8 columns.  64 target rows x WAVES waves per block; the
//            waves split the kernel evaluations of a 32-source tile, share
//            them through LDS, and each wave multiplies the whole tile into
//            its own group of nrp/WAVES columns.
//   mfma   : nrp >= 16 columns.  The column contraction runs on the FP64
//            matrix cores (see sweep_mfma).
// Sources are split into chunks (grid.y) so that large problems fill the
// chip; per-chunk partial sums are reduced in a fixed order (deterministic).
#include "sweep_pair.hpp"

namespace dp {

template <int OP, int NR>
__global__ __launch_bounds__(256) void sweep_private(SweepParams p) {
  constexpr int ND = Nd<OP>::v;
  const int n = p.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const int j0 = blockIdx.y * p.chunk_len;
  const int j1 = min(n, j0 + p.chunk_len);
  cplx acc[ND][NR];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[d][c] = {0.0, 0.0};
  int k = ii - j0;
  k += (k < 0) ? n : 0;
  for (int j = j0; j < j1; ++j) {
    const SrcRec s = p.src[j];
    const double Ck = p.C[k];
    cplx K[ND];
    pair_kernel_far<OP>(t, s, Ck, ii == j, p.omega, p.eta, p.dt, p.r2near, K);
    const cplx* dj = p.dens + (size_t)j * ND * NR;
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int c = 0; c < NR; ++c) cfma(acc[d][c], K[d], dj[d * NR + c]);
    k = (k == 0) ? n - 1 : k - 1;
  }
  if (i < n) {
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int c = 0; c < NR; ++c)
        p.partial[(((size_t)blockIdx.y * ND + d) * NR + c) * n + i] = acc[d][c];
  }
}

template <int OP, int NRG, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void sweep_shared(SweepParams p) {
  constexpr int ND = Nd<OP>::v;
  constexpr int TJ = 32;
  constexpr int PER = TJ / WAVES;
  __shared__ cplx Ks[TJ][ND][64];
  const int n = p.n;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blockIdx.x * 64 + lane;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const int j0 = blockIdx.y * p.chunk_len;
  const int j1 = min(n, j0 + p.chunk_len);
  const int nrp = p.nrp;
  cplx acc[ND][NRG];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int c = 0; c < NRG; ++c) acc[d][c] = {0.0, 0.0};
  for (int jt = j0; jt < j1; jt += TJ) {
#pragma unroll 1
    for (int q = 0; q < PER; ++q) {
      const int jj = w * PER + q;
      const int j = jt + jj;
      cplx K[ND];
      if (j < j1) {
        int k = ii - j;
        k += (k < 0) ? n : 0;
        pair_kernel_far<OP>(t, p.src[j], p.C[k], ii == j, p.omega, p.eta, p.dt, p.r2near, K);
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) K[d] = {0.0, 0.0};
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) Ks[jj][d][lane] = K[d];
    }
    __syncthreads();
    const int jn = min(TJ, j1 - jt);
    for (int jj = 0; jj < jn; ++jj) {
      const cplx* dj = p.dens + (size_t)(jt + jj) * ND * nrp + w * NRG;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const cplx Kv = Ks[jj][d][lane];
#pragma unroll
        for (int c = 0; c < NRG; ++c) cfma(acc[d][c], Kv, dj[d * nrp + c]);
      }
    }
    __syncthreads();
  }
  if (i < n) {
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int c = 0; c < NRG; ++c)
        p.partial[(((size_t)blockIdx.y * ND + d) * nrp + w * NRG + c) * n + i] = acc[d][c];
  }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Precision traits of the matrix-core sweep.  FP64: v_mfma_f64_16x16x4,
// result D[i][c] in register r of lane c + 16 (i mod 4), i = 4r + lane/16.
// FP32: v_mfma_f32_16x16x4 (FP32 products and accumulation within a source
// chunk), result D[i][c] in register r of lane c + 16 (i / 4),
// i = 4 (lane/16) + r.  Either way A[i][k] sits in lane i + 16k and
// B[k][c] in lane c + 16k.
struct Mfma64 {
  using C = cplx;
  using V4 = dbl4;
  static __device__ __forceinline__ V4 mma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
  static __device__ __forceinline__ const C* dens(const SweepParams& p) { return p.dens; }
  static __device__ __forceinline__ C* partial(const SweepParams& p) { return p.partial; }
  template <int OP>
  static __device__ __forceinline__ void far(const Tgt& t, const SrcRec& s, double Ck, bool self,
                                             const SweepParams& p, C* K) {
    pair_kernel_far<OP>(t, s, Ck, self, p.omega, p.eta, p.dt, p.r2near, K);
  }
};

struct Mfma32 {
  using C = cplxf;
  using V4 = flt4;
  static __device__ __forceinline__ V4 mma(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
  static __device__ __forceinline__ const C* dens(const SweepParams& p) { return p.dens32; }
  static __device__ __forceinline__ C* partial(const SweepParams& p) { return p.partial32; }
  template <int OP>
  static __device__ __forceinline__ void far(const Tgt& t, const SrcRec& s, double Ck, bool self,
                                             const SweepParams& p, C* K) {
    pair_kernel_far32<OP>(t, s, Ck, self, p.omega, p.eta, p.r2near, K);
  }
};

// Many-column sweep on the matrix cores.  The contraction
//   out_d[i][c] += sum_j K_d(i, j) dens_d[j][c]
// is a dense complex GEMM whose left operand is generated on the fly: a
// 16 x 4 tile of kernel values (16 targets x 4 sources, one pair per lane)
// is the A operand of a 16x16x4 MFMA, and the densities of the same 4
// sources for 16 columns are its B operand.
// Block: 8 waves = 4 row groups (16 targets each) x 2 column halves.  The
// two waves of a row group evaluate alternate 4-source steps and swap their
// kernel values through a double-buffered LDS slot (one barrier per pair of
// steps), so every kernel value is computed once per block; each wave then
// multiplies both steps into its own half of the columns.
// The densities of a pair of steps (8 sources x ND x NC columns, one
// contiguous run of the packed array) are staged once per block in a
// double-buffered LDS tile, with the sums re + im that the 3-multiplication
// products need: the block's threads request the next pair's tile
// before the kernel evaluation and store it after the barrier, so the load
// latency hides behind the evaluation and the four row groups share one copy.
// The source record and C_k of a wave's next step are prefetched the same way.
// Complex products take three real MFMAs: T1 += Kr Br, T2 += Ki Bi,
// T3 += (Kr + Ki)(Br + Bi); Re = T1 - T2, Im = T3 - T1 - T2.
template <int OP, int NCBW, class M>
__global__ __launch_bounds__(512) void sweep_mfma(SweepParams p) {
  using C = typename M::C;
  using V4 = typename M::V4;
  using R = decltype(C{}.re);
  constexpr int ND = Nd<OP>::v;
  constexpr int NC = 32 * NCBW;            // columns of the block = nrp (two waves per row group)
  constexpr int TILE = 8 * ND * NC;        // density tile of a pair of steps
  constexpr int PER = (TILE + 511) / 512;  // tile elements per thread
  __shared__ C Kx[2][4][2][ND][64];        // [buffer][row group][step parity][density][lane]
  __shared__ C Bt[2][TILE];                // [buffer][(source * ND + density) * NC + column]
  __shared__ R Bs[2][TILE];                // re + im of the same entries (3-multiplication products)
  const int n = p.n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int rg = wv & 3;                   // row group: 16 targets
  const int ch = wv >> 2;                  // column half; also the parity of the k-steps it evaluates
  const int c0 = ch * 16 * NCBW;
  const int li = lane & 15, lk = lane >> 4;
  const int i = blockIdx.x * 64 + rg * 16 + li;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const int j0 = blockIdx.y * p.chunk_len;
  const int j1 = min(n, j0 + p.chunk_len);
  const int nsteps = (j1 - j0 + 3) / 4;
  const int npairs = (nsteps + 1) / 2;
  const C* dens = M::dens(p);
  // Tile rows past the chunk are clamped to its last source (finite values
  // that meet zero kernel values).  Every thread issues exactly PER loads
  // (indices clamped into the tile, extra elements discarded at the store)
  // so the number of loads in flight is the same on every path and the
  // compiler's wait counts stay partial.
  auto load_tile = [&](int sp, C* reg) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = min(tid + 512 * q, TILE - 1);
      const int jr = e / (ND * NC);
      const int j = min(j0 + 8 * sp + jr, j1 - 1);
      reg[q] = dens[(size_t)j * ND * NC + (e - jr * ND * NC)];
    }
  };
  auto store_tile = [&](int buf, const C* reg) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 512 * q;
      if (e < TILE) {
        Bt[buf][e] = reg[q];
        Bs[buf][e] = reg[q].re + reg[q].im;
      }
    }
  };
  V4 T1[ND][NCBW], T2[ND][NCBW], T3[ND][NCBW];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int cb = 0; cb < NCBW; ++cb) {
      T1[d][cb] = V4{0, 0, 0, 0};
      T2[d][cb] = V4{0, 0, 0, 0};
      T3[d][cb] = V4{0, 0, 0, 0};
    }
  // source of this wave's k-step st: j = j0 + 4 st + lk (clamped into the chunk)
  auto src_of = [&](int st, int& jc, int& k) {
    jc = min(j0 + 4 * st + lk, j1 - 1);
    k = ii - jc;
    k += (k < 0) ? n : 0;
  };
  C breg[PER];
  load_tile(0, breg);
  store_tile(0, breg);  // read after the first barrier
  int jc, k;
  src_of(ch, jc, k);
  SrcRec sr = p.src[jc];
  double Ck = p.C[k];
  for (int sp = 0; sp < npairs; ++sp) {
    const int st = 2 * sp + ch;
    const bool valid = j0 + 4 * st + lk < j1;
    const bool self = ii == jc;
    const bool more = sp + 1 < npairs;
    load_tile(sp + 1, breg);  // past the last pair: clamped rows, never stored
    int jn, kn;
    src_of(st + 2, jn, kn);  // clamped: the last iteration reloads a valid record
    const SrcRec srn = p.src[jn];
    const double Ckn = p.C[kn];

    C K[ND];
    M::template far<OP>(t, sr, Ck, self, p, K);
    const int buf = sp & 1;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      K[d] = valid ? K[d] : C{0, 0};
      Kx[buf][rg][ch][d][lane] = K[d];
    }
    __syncthreads();
    // every wave has left the previous pair's products: its tile buffer is free
    if (more) store_tile(buf ^ 1, breg);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (2 * sp + h >= nsteps) break;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const C Kh = (h == ch) ? K[d] : Kx[buf][rg][h][d][lane];
        const R ks = Kh.re + Kh.im;
        const int o = ((4 * h + lk) * ND + d) * NC + c0 + li;
#pragma unroll
        for (int cb = 0; cb < NCBW; ++cb) {
          const C Bv = Bt[buf][o + cb * 16];
          T1[d][cb] = M::mma(Kh.re, Bv.re, T1[d][cb]);
          T2[d][cb] = M::mma(Kh.im, Bv.im, T2[d][cb]);
          T3[d][cb] = M::mma(ks, Bs[buf][o + cb * 16], T3[d][cb]);
        }
      }
    }
    sr = srn;
    Ck = Ckn;
    jc = jn;
  }
  C* part = M::partial(p);
  const int rbase = blockIdx.x * 64 + rg * 16;
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int cb = 0; cb < NCBW; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rbase + M::row(r, lk);
        if (row < n) {
          const R t1 = T1[d][cb][r], t2 = T2[d][cb][r], t3 = T3[d][cb][r];
          part[(((size_t)blockIdx.y * ND + d) * NC + c0 + cb * 16 + li) * n + row] = C{t1 - t2, t3 - t1 - t2};
        }
      }
}

// ------------------------------------------------------------ mixed precision
// Private shape with FP32 kernel values; the few products per pair are
// accumulated in FP64 (FP64 and FP32 VALU issue at the same rate here).
template <int OP, int NR>
__global__ __launch_bounds__(256) void sweep_private32(SweepParams p) {
  constexpr int ND = Nd<OP>::v;
  const int n = p.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const int j0 = blockIdx.y * p.chunk_len;
  const int j1 = min(n, j0 + p.chunk_len);
  cplx acc[ND][NR];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[d][c] = {0.0, 0.0};
  int k = ii - j0;
  k += (k < 0) ? n : 0;
  for (int j = j0; j < j1; ++j) {
    const SrcRec s = p.src[j];
    const double Ck = p.C[k];
    cplxf K[ND];
    pair_kernel_far32<OP>(t, s, Ck, ii == j, p.omega, p.eta, p.r2near, K);
    const cplx* dj = p.dens + (size_t)j * ND * NR;
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int c = 0; c < NR; ++c) cfma(acc[d][c], cplx{(double)K[d].re, (double)K[d].im}, dj[d * NR + c]);
    k = (k == 0) ? n - 1 : k - 1;
  }
  if (i < n) {
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int c = 0; c < NR; ++c)
        p.partial[(((size_t)blockIdx.y * ND + d) * NR + c) * n + i] = acc[d][c];
  }
}

// dens[j][d][c] = in_d[c*n + j] (zero for padded columns c >= nrhs), FP32
__global__ void pack_dens32(const cplx* __restrict__ a, const cplx* __restrict__ b, cplxf* __restrict__ dens,
                            int n, int nrhs, int nrp, int nd, int col0) {
  const size_t tot = (size_t)n * nrp * nd;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = idx % nrp;
    const int d = (idx / nrp) % nd;
    const size_t j = idx / ((size_t)nrp * nd);
    const cplx* src = d == 0 ? a : b;
    const cplx v = (c < nrhs) ? src[(size_t)(col0 + c) * n + j] : cplx{0.0, 0.0};
    dens[idx] = {(float)v.re, (float)v.im};
  }
}

// dens[j][d][c] = in_d[c*n + j] (zero for padded columns c >= nrhs)
__global__ void pack_dens(const cplx* __restrict__ a, const cplx* __restrict__ b, cplx* __restrict__ dens,
                          int n, int nrhs, int nrp, int nd, int col0) {
  const size_t tot = (size_t)n * nrp * nd;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = idx % nrp;
    const int d = (idx / nrp) % nd;
    const size_t j = idx / ((size_t)nrp * nd);
    const cplx* src = d == 0 ? a : b;
    dens[idx] = (c < nrhs) ? src[(size_t)(col0 + c) * n + j] : cplx{0.0, 0.0};
  }
}

// y = 1/2 q + v + w/(i eta)
__global__ void hard_combine(const cplx* __restrict__ q, const cplx* __restrict__ v,
                             const cplx* __restrict__ w, cplx* __restrict__ y, size_t tot, double eta) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const cplx a = q[idx], b = v[idx], c = w[idx];
    // c/(i eta) = -i c/eta
    y[idx] = {0.5 * a.re + b.re + c.im / eta, 0.5 * a.im + b.im - c.re / eta};
  }
}

static int grid1d(size_t tot) {
  size_t g = (tot + 255) / 256;
  return (int)(g > 8192 ? 8192 : (g ? g : 1));
}

template <int OP>
static void launch_sweep(const SweepParams& sp, int nrp, hipStream_t st) {
  const int n = sp.n;
  if (nrp <= 4) {
    dim3 grid((n + 255) / 256, sp.nchunks);
    switch (nrp) {
      case 1: sweep_private<OP, 1><<<grid, 256, 0, st>>>(sp); break;
      case 2: sweep_private<OP, 2><<<grid, 256, 0, st>>>(sp); break;
      default: sweep_private<OP, 4><<<grid, 256, 0, st>>>(sp); break;
    }
  } else {
    dim3 grid((n + 63) / 64, sp.nchunks);
    switch (nrp) {
      case 8: sweep_shared<OP, 2, 4><<<grid, 256, 0, st>>>(sp); break;
      case 16: sweep_shared<OP, 4, 4><<<grid, 256, 0, st>>>(sp); break;
      case 32: sweep_mfma<OP, 1, Mfma64><<<grid, 512, 0, st>>>(sp); break;
      default: sweep_mfma<OP, 2, Mfma64><<<grid, 512, 0, st>>>(sp); break;
    }
  }
}

template <int OP>
static void launch_sweep32(const SweepParams& sp, int nrp, hipStream_t st) {
  const int n = sp.n;
  if (nrp <= 4) {
    dim3 grid((n + 255) / 256, sp.nchunks);
    switch (nrp) {
      case 1: sweep_private32<OP, 1><<<grid, 256, 0, st>>>(sp); break;
      case 2: sweep_private32<OP, 2><<<grid, 256, 0, st>>>(sp); break;
      default: sweep_private32<OP, 4><<<grid, 256, 0, st>>>(sp); break;
    }
  } else {
    dim3 grid((n + 63) / 64, sp.nchunks);
    if (nrp == 32) sweep_mfma<OP, 1, Mfma32><<<grid, 512, 0, st>>>(sp);
    else sweep_mfma<OP, 2, Mfma32><<<grid, 512, 0, st>>>(sp);
  }
}

static int pad_cols(int nrhs) {
  int r = 1;
  while (r < nrhs && r < 64) r *= 2;
  return r;
}

static int tune_key(int prec, int op, int nrp) { return prec * 1000 + op * 100 + nrp; }

// Core sweep over one group of <= 64 columns.  a (and b for hard) are the
// densities; results go to out0 (and out1).
static int sweep_group(dp_problem* p, int op, int nrhs, int col0, const cplx* a, const cplx* b,
                       cplx* out0, cplx* out1, int prec) {
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n;
  const int nd = op == OP_HARD ? 2 : 1;
  int nrp = pad_cols(nrhs);
  dp_problem::SweepCfg cfg;
  {
    const auto it = p->tuned.find(tune_key(prec, op, nrp));
    if (it != p->tuned.end()) cfg = it->second;
  }
  // matrix-core shape for every multi-column mixed sweep, and for FP64 sweeps
  // of 8-16 columns when the autotuner found it faster than the VALU kernel
  if (nrp > 4 && nrp < 32 && (prec || cfg.mfma == 1)) nrp = 32;
  const bool part32 = prec && nrp > 4;
  const int rows_per_block = nrp <= 4 ? 256 : 64;
  const int bx = (n + rows_per_block - 1) / rows_per_block;
  int nchunks = (cfg.target_blocks + bx - 1) / bx;
  int maxch = n / 64 > 0 ? n / 64 : 1;
  if (nchunks > maxch) nchunks = maxch;
  if (nchunks < 1) nchunks = 1;
  int chunk_len = (n + nchunks - 1) / nchunks;
  if (nrp > 4) chunk_len = (chunk_len + 31) / 32 * 32;
  nchunks = (n + chunk_len - 1) / chunk_len;
  DP_TRY(p->dens.reserve((size_t)n * nrp * nd * sizeof(cplx)));
  DP_TRY(p->partial.reserve((size_t)nchunks * nd * nrp * n * sizeof(cplx)));
  {
    size_t tot = (size_t)n * nrp * nd;
    if (part32)
      pack_dens32<<<grid1d(tot), 256, 0, st>>>(a, b, reinterpret_cast<cplxf*>(p->dens.p), n, nrhs, nrp, nd, col0);
    else
      pack_dens<<<grid1d(tot), 256, 0, st>>>(a, b, p->dens.as<cplx>(), n, nrhs, nrp, nd, col0);
  }
  SweepParams sp;
  sp.src = p->src.as<SrcRec>();
  sp.C = p->C.as<double>();
  sp.dens = p->dens.as<cplx>();
  sp.partial = p->partial.as<cplx>();
  sp.dens32 = reinterpret_cast<const cplxf*>(p->dens.p);
  sp.partial32 = reinterpret_cast<cplxf*>(p->partial.p);
  sp.n = n;
  sp.nrp = nrp;
  sp.nd = nd;
  sp.chunk_len = chunk_len;
  sp.nchunks = nchunks;
  sp.omega = p->omega;
  sp.eta = p->eta;
  sp.dt = 2.0 * kPi / n;
  sp.r2near = p->r2near;
  SweepClock& clk = prec ? p->clock32 : p->clock;
  clk.start(st);
  if (prec) {
    switch (op) {
      case OP_SOFT: launch_sweep32<OP_SOFT>(sp, nrp, st); break;
      case OP_HARD: launch_sweep32<OP_HARD>(sp, nrp, st); break;
      case OP_S: launch_sweep32<OP_S>(sp, nrp, st); break;
      case OP_D: launch_sweep32<OP_D>(sp, nrp, st); break;
      default: launch_sweep32<OP_DP>(sp, nrp, st); break;
    }
  } else {
    switch (op) {
      case OP_SOFT: launch_sweep<OP_SOFT>(sp, nrp, st); break;
      case OP_HARD: launch_sweep<OP_HARD>(sp, nrp, st); break;
      case OP_S: launch_sweep<OP_S>(sp, nrp, st); break;
      case OP_D: launch_sweep<OP_D>(sp, nrp, st); break;
      default: launch_sweep<OP_DP>(sp, nrp, st); break;
    }
  }
  clk.stop(st);
  DP_HIP(hipGetLastError());
  DP_TRY(near_apply_group(p, op, nrp, p->dens.p, part32));
  EpiParams e;
  e.src = sp.src;
  e.partial = sp.partial;
  e.nearp = p->near_nnz > 0 ? p->near_out.as<cplx>() : nullptr;
  e.q = op == OP_HARD ? b : a;
  e.q2 = op == OP_HARD ? a : nullptr;
  e.out0 = out0;
  e.out1 = out1;
  e.n = n;
  e.nrhs = nrhs;
  e.nrp = nrp;
  e.nchunks = nchunks;
  e.op = op;
  e.col0 = col0;
  e.omega = p->omega;
  e.eta = p->eta;
  e.dt = sp.dt;
  e.R0 = p->R0;
  if (part32) sweep_epilogue<cplxf><<<grid1d((size_t)n * nrhs), 256, 0, st>>>(e);
  else sweep_epilogue<cplx><<<grid1d((size_t)n * nrhs), 256, 0, st>>>(e);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

// Time whole single-group sweeps (packing, sweep, near field, epilogue) of
// this problem's operator over the candidate launch configurations and keep
// the fastest for (precision, operator, column count).  The configuration
// changes the order in which partial sums are added, so results are
// reproducible for a given configuration, which stays fixed once chosen.
int autotune(dp_problem* p, int nrhs, int prec, dp_tune_info* info) {
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n;
  const int op = p->kind == DP_HARD ? OP_HARD : OP_SOFT;
  const int ng = nrhs < 64 ? nrhs : 64;
  const int nrp = pad_cols(ng);
  const int key = tune_key(prec, op, nrp);
  const size_t bytes = (size_t)n * ng * sizeof(cplx);
  DevBuf a, b, o0, o1;
  DP_TRY(a.reserve(bytes));
  DP_TRY(b.reserve(bytes));
  DP_TRY(o0.reserve(bytes));
  DP_TRY(o1.reserve(bytes));
  DP_HIP(hipMemsetAsync(a.p, 0, bytes, st));
  DP_HIP(hipMemsetAsync(b.p, 0, bytes, st));
  std::vector<dp_problem::SweepCfg> cands;
  const int modes = (!prec && (nrp == 8 || nrp == 16)) ? 2 : 1;
  for (int mode = 0; mode < modes; ++mode)
    for (int tb : {1024, 2048, 4096, 8192}) {
      dp_problem::SweepCfg c;
      c.target_blocks = tb;
      c.mfma = modes == 2 ? mode : -1;
      cands.push_back(c);
    }
  hipEvent_t e0, e1;
  DP_HIP(hipEventCreate(&e0));
  DP_HIP(hipEventCreate(&e1));
  double best = 1e30, t_default = 0;
  dp_problem::SweepCfg bestc;
  int rc = DP_OK;
  for (const auto& c : cands) {
    p->tuned[key] = c;
    double t = 1e30;
    for (int rep = 0; rep < 3 && rc == DP_OK; ++rep) {
      (void)hipEventRecord(e0, st);
      rc = sweep_group(p, op, ng, 0, a.as<cplx>(), b.as<cplx>(), o0.as<cplx>(), o1.as<cplx>(), prec);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) rc = DP_EDEVICE;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) t = std::min(t, (double)ms);  // the first run also allocates
    }
    if (rc != DP_OK) break;
    if (c.target_blocks == 2048 && c.mfma <= 0) t_default = t;
    if (t < best) {
      best = t;
      bestc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->clock.reset();
  p->clock32.reset();
  a.release();
  b.release();
  o0.release();
  o1.release();
  if (rc != DP_OK) {
    p->tuned.erase(key);
    return rc;
  }
  p->tuned[key] = bestc;
  if (info) {
    info->t_default_ms = t_default;
    info->t_best_ms = best;
    info->target_blocks = bestc.target_blocks;
    info->matrix_cores = bestc.mfma == 1 || (prec && nrp > 4) || nrp >= 32 ? 1 : 0;
    info->candidates = (int64_t)cands.size();
  }
  return DP_OK;
}

void SweepClock::start(hipStream_t s) {
  if (used + 2 > ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    ev.push_back(a);
    ev.push_back(b);
  }
  (void)hipEventRecord(ev[used], s);
}

void SweepClock::stop(hipStream_t s) {
  if (used + 2 > ev.size()) return;
  (void)hipEventRecord(ev[used + 1], s);
  used += 2;
}

void SweepClock::collect() {
  for (size_t k = 0; k + 1 < used; k += 2) {
    float ms = 0.f;
    if (hipEventSynchronize(ev[k + 1]) == hipSuccess && hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) {
      seconds += 1e-3 * ms;
      ++launches;
    }
  }
  used = 0;
}

void SweepClock::destroy() {
  for (auto e : ev) (void)hipEventDestroy(e);
  ev.clear();
  used = 0;
}

int sweep_apply(dp_problem* p, int op, int nrhs, const cplx* q, cplx* y, int prec) {
  for (int c0 = 0; c0 < nrhs; c0 += 64) {
    const int nc = nrhs - c0 < 64 ? nrhs - c0 : 64;
    DP_TRY(sweep_group(p, op, nc, c0, q, nullptr, y, nullptr, prec));
  }
  return DP_OK;
}

int matvec(dp_problem* p, int nrhs, const cplx* q, cplx* y, int prec) {
  if (p->kind == DP_SOFT) return sweep_apply(p, OP_SOFT, nrhs, q, y, prec);
  const size_t tot = (size_t)p->n * nrhs;
  DP_TRY(p->tmp1.reserve(tot * sizeof(cplx)));
  DP_TRY(p->tmp2.reserve(tot * sizeof(cplx)));
  DP_TRY(p->tmp3.reserve(tot * sizeof(cplx)));
  cplx* sig = p->tmp1.as<cplx>();
  cplx* u = p->tmp2.as<cplx>();
  cplx* v = p->tmp3.as<cplx>();
  DP_TRY(spectral_derivative(p, nrhs, q, sig));
  for (int c0 = 0; c0 < nrhs; c0 += 64) {
    const int nc = nrhs - c0 < 64 ? nrhs - c0 : 64;
    DP_TRY(sweep_group(p, OP_HARD, nc, c0, sig, q, u, v, prec));
  }
  DP_TRY(spectral_derivative(p, nrhs, u, sig));
  hard_combine<<<grid1d(tot), 256, 0, p->ctx->stream>>>(q, v, sig, y, tot, p->eta);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

}  // namespace dp
