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
//            matrix cores (see sweep_mfma); single precision: split-FP16
//            operands on the FP16 matrix cores (see sweep_mfma16).
// Sources are split into chunks (grid.y) so that large problems fill the
// chip; per-chunk partial sums are reduced in a fixed order (deterministic).
#include <algorithm>
#include <cmath>

#include "sweep_pair.hpp"

namespace dp {

// A launch queued for an Arnoldi step after every column stopped does no
// work: the guard flags are read once per block (uniform scalar loads), and
// the whole block returns before any barrier.
__device__ __forceinline__ bool sweep_skipped(const SweepParams& p) {
  if (!p.guard) return false;
  int any = 0;
  for (int c = 0; c < p.guard_n; ++c) any |= p.guard[c];
  return any == 0;
}

template <int OP, int NR>
__global__ __launch_bounds__(256) void sweep_private(SweepParams p) {
  if (sweep_skipped(p)) return;
  constexpr int ND = Nd<OP>::v;
  const int n = p.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const Far32 f = far32_consts(p.omega, p.eta, p.r2near, 1.0f, 1.0f);
  const Tgt32 tf = tgt32<OP>(tr.nx, tr.ny, f);
  const double rho_scale = 1.0 / (kPi * p.dt);  // rho = C_k / (pi dt)
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
  if (sweep_skipped(p)) return;
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

// Precision traits of the FP64 matrix-core sweep: v_mfma_f64_16x16x4,
// A[i][k] in lane i + 16k, B[k][c] in lane c + 16k, result D[i][c] in
// register r of lane c + 16 (i mod 4), i = 4r + lane/16.
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
// SPLITK (16 columns): both waves of a row group take all 16 columns but only
// the steps they evaluate themselves (no kernel values change hands), and
// their sums are added through LDS at the end: half the products of the
// 32-column shape padded from 16.
template <int OP, int NCBW, class M, bool SPLITK = false>
__global__ __launch_bounds__(512) void sweep_mfma(SweepParams p) {
  if (sweep_skipped(p)) return;
  using C = typename M::C;
  using V4 = typename M::V4;
  using R = decltype(C{}.re);
  constexpr int ND = Nd<OP>::v;
  static_assert(!SPLITK || NCBW == 1, "the split-k shape has one 16-column tile per wave");
  constexpr int NC = SPLITK ? 16 : 32 * NCBW;  // columns of the block = nrp
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
  const int c0 = SPLITK ? 0 : ch * 16 * NCBW;
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
      if (!SPLITK) Kx[buf][rg][ch][d][lane] = K[d];
    }
    __syncthreads();
    // every wave has left the previous pair's products: its tile buffer is free
    if (more) store_tile(buf ^ 1, breg);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (SPLITK && h != ch) continue;
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
  if constexpr (SPLITK) {
    // the second wave of each row group hands its complex sums
    // (T1 - T2, T3 - T1 - T2) to the first through the (now unused) exchange
    // buffer, [row group][d][r][re, im][lane]; the first adds them to its own
    // sums folded the same way (kept in T1 and T3)
    R* red = reinterpret_cast<R*>(&Kx[0][0][0][0][0]);
    static_assert(4 * ND * 4 * 2 * 64 * sizeof(R) <= sizeof(Kx), "exchange buffer too small");
    __syncthreads();
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const R t1 = T1[d][0][r], t2 = T2[d][0][r], t3 = T3[d][0][r];
        T1[d][0][r] = t1 - t2;
        T3[d][0][r] = t3 - t1 - t2;
        if (ch == 1) {
          R* o = red + ((rg * ND + d) * 4 + r) * 128 + lane;
          o[0] = t1 - t2;
          o[64] = t3 - t1 - t2;
        }
      }
    __syncthreads();
    if (ch == 1) return;
    C* part = M::partial(p);
    const int rbase = blockIdx.x * 64 + rg * 16;
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const R* o = red + ((rg * ND + d) * 4 + r) * 128 + lane;
        const int row = rbase + M::row(r, lk);
        if (row < n)
          part[(((size_t)blockIdx.y * ND + d) * NC + li) * n + row] = C{T1[d][0][r] + o[0], T3[d][0][r] + o[64]};
      }
    return;
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
  if (sweep_skipped(p)) return;
  constexpr int ND = Nd<OP>::v;
  const int n = p.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const Far32 f = far32_consts(p.omega, p.eta, p.r2near, 1.0f, 1.0f);
  const Tgt32 tf = tgt32<OP>(tr.nx, tr.ny, f);
  const double rho_scale = 1.0 / (kPi * p.dt);  // rho = C_k / (pi dt)
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
    cplxf K[ND];
    pair_kernel_far32<OP>(t, tf, s, (float)(p.C[k] * rho_scale), false, f, K);
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

// dens[j][d][c] = in_d[c*n + j] (zero for padded columns c >= nrhs), in
// FP64 (OT = cplx) or FP32 (OT = cplxf)
template <class OT>
__global__ __launch_bounds__(256) void pack_dens_t(const cplx* __restrict__ a, const cplx* __restrict__ b,
                                                   OT* __restrict__ dens, int n, int nrhs, int nrp, int nd,
                                                   int col0) {
  // block (32-row block, density): the 32 x nrp slab (nrp <= 64) is read
  // along the rows of each column, transposed through LDS and written along
  // the columns
  __shared__ OT tile[32][65];
  const int j0 = blockIdx.x * 32, d = blockIdx.y;
  const cplx* src = d == 0 ? a : b;
  for (int e = threadIdx.x; e < 32 * nrp; e += 256) {
    const int c = e >> 5, jj = e & 31;
    const int j = j0 + jj;
    const cplx v = (c < nrhs && j < n) ? src[(size_t)(col0 + c) * n + j] : cplx{0.0, 0.0};
    tile[jj][c] = OT{(decltype(OT{}.re))v.re, (decltype(OT{}.re))v.im};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * nrp; e += 256) {
    const int jj = e / nrp, c = e - jj * nrp;
    const int j = j0 + jj;
    if (j < n) dens[((size_t)j * nd + d) * nrp + c] = tile[jj][c];
  }
}

// ------------------------------------------------ split-FP16 matrix-core sweep
// The single-precision contraction on the FP16 matrix cores
// (v_mfma_f32_16x16x32_f16: 16 targets x 32 sources x 16 columns, FP32
// accumulation).  Both operands are scaled by powers of two and split as
// x = hi + lo with hi = fp16(x), lo = fp16(x - hi) (round toward zero); each
// real product takes hi*hi + hi*lo + lo*hi, which keeps about 21 bits of the
// FP32 operands, below the error of the FP32 kernel values themselves.
//   kernel values: scale 2^eK[d], fixed per problem and operator from a bound
//                  on the far-field values (|H0|, |H1| <= 0.25 for omega r >= 25);
//   densities    : scale 2^eB[d][c] per column, from the column's largest part.
// A complex product takes four real ones: Re += Kr Br + (-Ki) Bi,
// Im += Kr Bi + Ki Br.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// hi = fp16(a, b) and lo = fp16 of the remainders, both round toward zero
// (never overflows to infinity), packed two halves per word.
// x - h for the FP16 half `SEL` of h, as one mixed-precision FMA
// (x + (-h) * 1), or -x - h with NEG (the negation as a source modifier).
// With h = x rounded toward zero to FP16 the difference has at most 13
// significant bits, so it is exact in FP32.
template <int SEL, bool NEG>
__device__ __forceinline__ float sub_half(float x, uint32_t h) {
  float r;
  if constexpr (SEL == 0 && !NEG)
    asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
  else if constexpr (SEL == 0)
    asm("v_fma_mix_f32 %0, -%1, 1.0, -%2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
  else if constexpr (!NEG)
    asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
  else
    asm("v_fma_mix_f32 %0, -%1, 1.0, -%2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
  return r;
}

// hi = FP16 pair (a, b) rounded toward zero, lo = FP16 pair of the
// remainders; with NEG the pair split is (-a, -b).
template <bool NEG = false>
__device__ __forceinline__ void split_h2(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, NEG ? __builtin_amdgcn_cvt_pkrtz(-a, -b) : __builtin_amdgcn_cvt_pkrtz(a, b));
  lo = __builtin_bit_cast(uint32_t,
                          __builtin_amdgcn_cvt_pkrtz(sub_half<0, NEG>(a, hi), sub_half<1, NEG>(b, hi)));
}

__device__ __forceinline__ flt4 mma16(const uint32_t (&a)[4], const uint4& b, flt4 c) {
  const uint4 av = {a[0], a[1], a[2], a[3]};
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, av), __builtin_bit_cast(half8, b), c,
                                                0, 0, 0);
}

// Density tiles: for each block of 32 sources b, density d, part
// (re hi, re lo, im hi, im lo) and column c, the 32 halves of the block's
// sources, i.e. uint4 index (((b * nd + d) * 4 + part) * nrp + c) * 4 + g for
// the 8 sources 32 b + 4 e + g, e = 0..7 (the contraction index 8 g + e
// stands for source 4 e + g).  Sources past n and columns past nrhs are zero.
// Block: 8 waves, each 16 targets x all nrp columns; per 32-source step
// every lane evaluates 8 pairs (target lane % 16, sources 4 e + lane / 16),
// which is exactly its A fragment; the four lane groups then read adjacent
// 16-byte records of the step's source block (positions, then FP32 normal
// and weight), on distinct LDS banks.  The step's density tile, its source
// block and the C_k window of the block (FP32 table of C_k / (pi dt)) reach LDS
// by direct global-to-LDS loads issued two steps ahead; the steps cycle
// through four separate sets of LDS arrays, so that reads of one set never
// wait for the loads into another, and the block synchronises after every
// second step (the loads for the next two steps are then complete, and the
// two sets they overwrite have been read).  In LDS the
// tile row (d, part, c) holds its four 16-byte chunks g at positions
// g ^ ((row / 4 ^ (row & 2)) % 4): the 16 lanes that read one chunk of 16
// consecutive rows land on 16 distinct 16-byte bank groups of 256 bytes,
// and each 8 consecutive lanes on 8 distinct ones of 128 bytes.
template <int OP, int NCB>
__global__ __launch_bounds__(512) void sweep_mfma16(SweepParams p) {
  if (sweep_skipped(p)) return;
  constexpr int ND = Nd<OP>::v;
  constexpr int NC = 16 * NCB;
  constexpr int TQ = ND * 4 * NC * 4;      // uint4 per tile
  constexpr int NQ = TQ / 64;              // wave loads per tile
  __shared__ uint4 Bt0[TQ], Bt1[TQ], Bt2[TQ], Bt3[TQ];
  __shared__ uint4 Ss0[64], Ss1[64], Ss2[64], Ss3[64];  // source block: 32 (x, y), 32 (nx, ny, w/4, 0)
  __shared__ float Cs0[192], Cs1[192], Cs2[192], Cs3[192];  // C_k for k = kb .. kb + 159 (mod n)
  const int n = p.n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = blockIdx.x * 128;
  const int ti = wv * 16 + li;             // target within the block
  const int i = i0 + ti;
  const int ii = i < n ? i : n - 1;
  const SrcRec tr = p.src[ii];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  const Far32 f = far32_consts(p.omega, p.eta, p.r2near, p.ksc[0], p.ksc[1]);
  const Tgt32 tf = tgt32<OP>(tr.nx, tr.ny, f);
  const int j0 = blockIdx.y * p.chunk_len;  // multiple of 32
  const int j1 = min(n, j0 + p.chunk_len);
  const int nsteps = (j1 - j0 + 31) / 32;
  const int gsw = lk ^ (((li >> 2) ^ (li & 2)) & 3);  // swizzled chunk of this lane's B fragments
  // wave-uniform direct loads of step st into one buffer set
  auto dma = [&](int st, uint4* Bt, uint4* Ss, float* Cs) {
    const int jb = j0 + 32 * st;
    const uint4* tile = p.dens16 + (size_t)(jb / 32) * TQ;
    for (int q = wv; q < NQ; q += 8) {
      const int P = 64 * q + lane;
      const int row = P >> 2;
      __builtin_amdgcn_global_load_lds(tile + row * 4 + ((P & 3) ^ (((row >> 2) ^ (row & 2)) & 3)), &Bt[64 * q], 16,
                                       0, 0);
    }
    if (wv == 7) {
      __builtin_amdgcn_global_load_lds(p.srcblk + (size_t)(jb / 32) * 64 + lane, Ss, 16, 0, 0);
    } else if (wv >= 3 && wv < 6) {
      const int P = 64 * (wv - 3) + lane;
      int k = (i0 - jb - 31 + min(P, 159)) % n;
      k += (k < 0) ? n : 0;
      __builtin_amdgcn_global_load_lds(p.C32 + k, &Cs[64 * (wv - 3)], 4, 0, 0);
    }
  };
  flt4 Re[ND][NCB], Im[ND][NCB];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      Re[d][cb] = flt4{0, 0, 0, 0};
      Im[d][cb] = flt4{0, 0, 0, 0};
    }
  auto step = [&](int st, const uint4* Bt, const uint4* Ss, const float* Cs, uint4* Btn, uint4* Ssn, float* Csn,
                  bool sync) {
    if (st + 2 < nsteps) dma(st + 2, Btn, Ssn, Csn);
    const int jb = j0 + 32 * st;
    const int lim = j1 - jb;  // sources at k-index jj >= lim lie past the chunk
    constexpr int CP = NCB >= 2 ? 2 : 1;
    constexpr int NG = NCB / CP;
    uint4 bb[2][CP][4];
    auto read_b = [&](int g, uint4 (&dst)[CP][4]) {
      const int d = g / NG, cb0 = (g % NG) * CP;
#pragma unroll
      for (int u = 0; u < CP; ++u) {
        const int row = d * 4 * NC + (cb0 + u) * 16 + li;
#pragma unroll
        for (int part = 0; part < 4; ++part) dst[u][part] = Bt[(row + part * NC) * 4 + gsw];
      }
    };
    // the first group's B fragments are requested before the pair
    // evaluation, so that they have arrived when its products start
    read_b(0, bb[0]);
    __builtin_amdgcn_sched_barrier(0);
    // A fragments: this lane's 8 pairs, hi and lo parts of Re K and Im K
    uint32_t arh[ND][4], arl[ND][4], aih[ND][4], ail[ND][4];
    const double2* sxy = reinterpret_cast<const double2*>(Ss);
    const float4* snw = reinterpret_cast<const float4*>(Ss + 32);
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
      cplxf K[2][ND];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jj = 4 * (2 * e2 + h) + lk;  // k-index 8 lk + e holds source 4 e + lk
        const double2 xy = sxy[jj];
        const float4 nw = snw[jj];
        // jj >= lim, with the step's constant part moved to the scalar side
        const bool past = lk >= lim - 4 * (2 * e2 + h);
        pair_kernel_far32v<OP>(t, tf, xy.x, xy.y, nw.x, nw.y, nw.z, Cs[31 + ti - jj], past, f, K[h]);
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        // the S-type value's real part is -A0 (pair_kernel_far32): split
        // it from A0 with the negation as a source modifier
        if (d == 0 && (OP == OP_S || OP == OP_HARD))
          split_h2<true>(-K[0][d].re, -K[1][d].re, arh[d][e2], arl[d][e2]);
        else
          split_h2(K[0][d].re, K[1][d].re, arh[d][e2], arl[d][e2]);
        split_h2(K[0][d].im, K[1][d].im, aih[d][e2], ail[d][e2]);
      }
    }
    // Products, in groups of two column blocks (four independent
    // accumulation chains) over (d, column pair); each group's B fragments
    // are read from LDS one group ahead, while the previous group's products
    // run (the scheduling barriers keep the reads from being hoisted into
    // one batch that would wait for all of them).
#pragma unroll
    for (int g = 0; g < ND * NG; ++g) {
      const int d = g / NG, cb0 = (g % NG) * CP;
      if (g + 1 < ND * NG) read_b(g + 1, bb[(g + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
      uint32_t nih[4], nil[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        nih[e] = aih[d][e] ^ 0x80008000u;
        nil[e] = ail[d][e] ^ 0x80008000u;
      }
      const uint4 (&B)[CP][4] = bb[g & 1];
      flt4 r[CP], m[CP];
#pragma unroll
      for (int u = 0; u < CP; ++u) {
        r[u] = Re[d][cb0 + u];
        m[u] = Im[d][cb0 + u];
      }
      // parts: 0 re hi, 1 re lo, 2 im hi, 3 im lo
#define DP_MMA2(AR, PR, AI, PI)                    \
  _Pragma("unroll") for (int u = 0; u < CP; ++u) { \
    r[u] = mma16(AR, B[u][PR], r[u]);              \
    m[u] = mma16(AI, B[u][PI], m[u]);              \
  }
      DP_MMA2(arh[d], 0, arh[d], 2)
      DP_MMA2(arh[d], 1, arh[d], 3)
      DP_MMA2(arl[d], 0, arl[d], 2)
      DP_MMA2(nih, 2, aih[d], 0)
      DP_MMA2(nih, 3, aih[d], 1)
      DP_MMA2(nil, 2, ail[d], 0)
#undef DP_MMA2
#pragma unroll
      for (int u = 0; u < CP; ++u) {
        Re[d][cb0 + u] = r[u];
        Im[d][cb0 + u] = m[u];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // after every second step: the loads of the next two steps are
    // complete and the reads of the two buffer sets they replace are done
    if (sync) __syncthreads();
  };
  dma(0, Bt0, Ss0, Cs0);
  if (nsteps > 1) dma(1, Bt1, Ss1, Cs1);
  __syncthreads();
  for (int st = 0; st < nsteps; st += 4) {
    step(st, Bt0, Ss0, Cs0, Bt2, Ss2, Cs2, false);
    if (st + 1 < nsteps) step(st + 1, Bt1, Ss1, Cs1, Bt3, Ss3, Cs3, true);
    if (st + 2 < nsteps) step(st + 2, Bt2, Ss2, Cs2, Bt0, Ss0, Cs0, false);
    if (st + 3 < nsteps) step(st + 3, Bt3, Ss3, Cs3, Bt1, Ss1, Cs1, true);
  }
  cplxf* part = p.partial32;
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = cb * 16 + li;
      const float us = p.unscale16[d * NC + c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wv * 16 + 4 * lk + r;
        if (row < n)
          part[(((size_t)blockIdx.y * ND + d) * NC + c) * n + row] = cplxf{Re[d][cb][r] * us, Im[d][cb][r] * us};
      }
    }
}

// Per-column power-of-two scales of the densities: one block per (d, c).
// eK: the kernel-value exponent of density d.  The density scale puts the
// column's largest |re| or |im| below 2^14; the combined exponent stays in
// [-120, 120] so that the FP32 unscale factor is a normal number.
__global__ __launch_bounds__(1024) void dens16_scales(const cplx* __restrict__ a, const cplx* __restrict__ b,
                                                      int n, int nrhs, int nrp, int col0, int eK0, int eK1,
                                                      double* __restrict__ bscale, float* __restrict__ unscale) {
  const int d = blockIdx.x / nrp, c = blockIdx.x % nrp;
  __shared__ double red[1024];
  double m = 0.0;
  if (c < nrhs) {
    const cplx* src = (d == 0 ? a : b) + (size_t)(col0 + c) * n;
    for (int j = threadIdx.x; j < n; j += 1024) {
      const cplx v = src[j];
      m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int eK = d == 0 ? eK0 : eK1;
    int eB = 0;
    if (red[0] > 0.0) {
      int e;
      (void)frexp(red[0], &e);  // red[0] < 2^e
      eB = 14 - e;
    }
    eB = max(eB, max(-100, -120 - eK));
    eB = min(eB, min(100, 120 - eK));
    bscale[blockIdx.x] = ldexp(1.0, eB);
    unscale[blockIdx.x] = (float)ldexp(1.0, -(eK + eB));
  }
}

// Split-FP16 density tiles (layout in sweep_mfma16); one thread per chunk
// (8 sources) of one (block, density, column).
__global__ void pack_dens16(const cplx* __restrict__ a, const cplx* __restrict__ b,
                            const double* __restrict__ bscale, uint4* __restrict__ out, int n, int nrhs,
                            int nrp, int nd, int col0, int nb) {
  const size_t tot = (size_t)nb * 4 * nd * nrp;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int g = idx & 3;
    const size_t bi = (idx >> 2) % nb;
    const int dc = (int)((idx >> 2) / nb);  // d * nrp + c
    const int d = dc / nrp, c = dc % nrp;
    const double sc = bscale[dc];
    const cplx* src = (d == 0 ? a : b) + (size_t)(col0 + c) * n;
    uint32_t rh[4], rl[4], ih[4], il[4];
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
      float v[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const size_t j = bi * 32 + 4 * (2 * e2 + h) + g;
        const cplx x = (c < nrhs && j < (size_t)n) ? src[j] : cplx{0.0, 0.0};
        v[h][0] = (float)(x.re * sc);
        v[h][1] = (float)(x.im * sc);
      }
      split_h2(v[0][0], v[1][0], rh[e2], rl[e2]);
      split_h2(v[0][1], v[1][1], ih[e2], il[e2]);
    }
    uint4* o = out + ((((bi * nd + d) * 4) * nrp + c) * 4 + g);
    const size_t ps = (size_t)nrp * 4;  // uint4 between parts
    o[0] = uint4{rh[0], rh[1], rh[2], rh[3]};
    o[ps] = uint4{rl[0], rl[1], rl[2], rl[3]};
    o[2 * ps] = uint4{ih[0], ih[1], ih[2], ih[3]};
    o[3 * ps] = uint4{il[0], il[1], il[2], il[3]};
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
static void launch_sweep(const SweepParams& sp, int nrp, hipStream_t st, bool mfma16 = false) {
  const int n = sp.n;
  if (mfma16) {  // 16 columns on the matrix cores, split over the k steps
    sweep_mfma<OP, 1, Mfma64, true><<<dim3((n + 63) / 64, sp.nchunks), 512, 0, st>>>(sp);
    return;
  }
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
    dim3 grid((n + 127) / 128, sp.nchunks);
    switch (nrp) {
      case 16: sweep_mfma16<OP, 1><<<grid, 512, 0, st>>>(sp); break;
      case 32: sweep_mfma16<OP, 2><<<grid, 512, 0, st>>>(sp); break;
      default: sweep_mfma16<OP, 4><<<grid, 512, 0, st>>>(sp); break;
    }
  }
}

// Exponents eK[d] of the power-of-two scales of the FP32 kernel values in the
// split-FP16 sweep: 2^eK times a bound on |Re K| and |Im K| of a far pair
// stays below 2^14.  For omega r >= 25, |H0| and |H1| are below 0.17; 0.25
// is used.  With w = dt |x'_j| and c = max_k |C_k| |x'_j|, the S-type part is
// at most 0.25 (w/4 + c/(4 pi)) and the D-type part omega times that.
static void kernel_scales(const dp_problem* p, int op, int eK[2]) {
  const double base = 0.25 * (0.25 * (2.0 * kPi / (double)p->n) * p->spmax + p->cmax * p->spmax * kInv4Pi);
  double bnd[2] = {base, base};
  switch (op) {
    case OP_SOFT: bnd[0] = (p->omega + p->eta) * base; break;
    case OP_S: break;
    case OP_D:
    case OP_DP: bnd[0] = p->omega * base; break;
    default: bnd[1] = (p->omega * p->omega / p->eta + p->omega) * base; break;
  }
  for (int d = 0; d < 2; ++d) {
    int e = 0;
    (void)std::frexp(bnd[d], &e);  // bnd < 2^e
    eK[d] = std::min(60, std::max(-60, 14 - e));
  }
}

static int pad_cols(int nrhs) {
  int r = 1;
  while (r < nrhs && r < 64) r *= 2;
  return r;
}

static int tune_key(int prec, int op, int nrp) { return prec * 1000 + op * 100 + nrp; }

// Launch configuration without tuning, from autotuner runs on random stars
// (n = 4096, 16384, 65536, soft and hard, 1-16 columns) and the 64-column
// kite at n = 32768:
//   <= 4 columns (one target row per lane): 8192 blocks from n = 16384 on
//     (7-20% faster than 2048), 4096 below;
//   FP64, 5-16 columns: the 16-column matrix-core kernel (split over the k
//     steps) on 1024 blocks for hard problems and for 16 columns up to
//     n = 32768, on 4096 blocks for 16 soft columns above (10-25% faster
//     than the VALU kernel), else the VALU kernel on 8192 blocks;
//   single precision, 5-16 columns: 1024 blocks up to n = 8192 (12%), 2048
//     above;
//   32-64 columns: 2048.
static dp_problem::SweepCfg default_cfg(const dp_problem* p, int prec, int op, int nrp) {
  dp_problem::SweepCfg c;
  const int64_t n = p->n;
  if (nrp <= 4) {
    c.target_blocks = n >= 16384 ? 8192 : 4096;
  } else if (nrp <= 16) {
    if (prec) {
      c.target_blocks = n <= 8192 ? 1024 : 2048;
    } else if ((op == OP_HARD && (nrp == 16 || n <= 32768)) || (nrp == 16 && n <= 32768)) {
      c.mfma = 1;
      c.target_blocks = 1024;
    } else if (nrp == 16) {
      c.mfma = 1;
      c.target_blocks = 4096;
    } else {
      c.mfma = 0;
      c.target_blocks = 8192;
    }
  }
  return c;
}

// Core sweep over one group of <= 64 columns.  a (and b for hard) are the
// densities; results go to out0 (and out1).
static int sweep_group(dp_problem* p, int op, int nrhs, int col0, const cplx* a, const cplx* b,
                       cplx* out0, cplx* out1, int prec) {
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n;
  const int nd = op == OP_HARD ? 2 : 1;
  int nrp = pad_cols(nrhs);
  dp_problem::SweepCfg cfg = default_cfg(p, prec, op, nrp);
  {
    const auto it = p->tuned.find(tune_key(prec, op, nrp));
    if (it != p->tuned.end()) cfg = it->second;
  }
  // matrix-core shape for every multi-column mixed sweep, and for FP64 sweeps
  // of 8-16 columns when the autotuner found it faster than the VALU kernel
  if (prec && nrp > 4 && nrp < 16) nrp = 16;
  const bool mfma16 = !prec && nrp > 4 && nrp <= 16 && cfg.mfma == 1;
  if (mfma16) nrp = 16;
  const bool part32 = prec && nrp > 4;
  const int rows_per_block = nrp <= 4 ? 256 : (part32 ? 128 : 64);
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
  int eK[2] = {0, 0};
  const int nb = (n + 31) / 32;
  if (part32) {
    kernel_scales(p, op, eK);
    DP_TRY(p->dens16.reserve((size_t)nb * nd * nrp * 256));
    DP_TRY(p->sc16.reserve((size_t)nd * nrp * (sizeof(double) + sizeof(float))));
  }
  double* bscale = p->sc16.as<double>();
  float* unscale = reinterpret_cast<float*>(bscale + nd * nrp);
  {
    if (part32) {
      pack_dens_t<cplxf><<<dim3((n + 31) / 32, nd), 256, 0, st>>>(a, b, reinterpret_cast<cplxf*>(p->dens.p), n,
                                                                 nrhs, nrp, nd, col0);
      dens16_scales<<<nd * nrp, 1024, 0, st>>>(a, b ? b : a, n, nrhs, nrp, col0, eK[0], eK[1], bscale, unscale);
      pack_dens16<<<grid1d((size_t)nb * 4 * nd * nrp), 256, 0, st>>>(a, b ? b : a, bscale, p->dens16.as<uint4>(),
                                                                      n, nrhs, nrp, nd, col0, nb);
    } else {
      pack_dens_t<cplx><<<dim3((n + 31) / 32, nd), 256, 0, st>>>(a, b, p->dens.as<cplx>(), n, nrhs, nrp, nd, col0);
    }
  }
  SweepParams sp;
  sp.src = p->src.as<SrcRec>();
  sp.srcblk = p->srcblk.as<uint4>();
  sp.C = p->C.as<double>();
  sp.C32 = p->C32.as<float>();
  sp.dens = p->dens.as<cplx>();
  sp.partial = p->partial.as<cplx>();
  sp.dens32 = reinterpret_cast<const cplxf*>(p->dens.p);
  sp.partial32 = reinterpret_cast<cplxf*>(p->partial.p);
  sp.dens16 = part32 ? p->dens16.as<uint4>() : nullptr;
  sp.unscale16 = part32 ? unscale : nullptr;
  sp.ksc[0] = std::ldexp(1.0f, eK[0]);
  sp.ksc[1] = std::ldexp(1.0f, eK[1]);
  sp.n = n;
  sp.nrp = nrp;
  sp.nd = nd;
  sp.chunk_len = chunk_len;
  sp.nchunks = nchunks;
  sp.omega = p->omega;
  sp.eta = p->eta;
  sp.dt = 2.0 * kPi / n;
  sp.r2near = p->r2near;
  sp.guard = p->sweep_guard;
  sp.guard_n = p->sweep_guard_n;
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
      case OP_SOFT: launch_sweep<OP_SOFT>(sp, nrp, st, mfma16); break;
      case OP_HARD: launch_sweep<OP_HARD>(sp, nrp, st, mfma16); break;
      case OP_S: launch_sweep<OP_S>(sp, nrp, st, mfma16); break;
      case OP_D: launch_sweep<OP_D>(sp, nrp, st, mfma16); break;
      default: launch_sweep<OP_DP>(sp, nrp, st, mfma16); break;
    }
  }
  clk.stop(st);
  DP_HIP(hipGetLastError());
  DP_TRY(near_apply_group(p, op, nrp, p->dens.p, part32));
  EpiParams e;
  e.src = sp.src;
  e.diag = p->diag.as<double4>();
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
    {
      const dp_problem::SweepCfg d = default_cfg(p, prec, op, nrp);
      if (c.target_blocks == d.target_blocks && (modes == 1 || c.mfma == (d.mfma == 1 ? 1 : 0))) t_default = t;
    }
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

// Diagonal (Kress limits) of S and of D = D' at every node:
//   S_ii = R0 (-sp/(4 pi)) + dt sp (i/4 - gamma/(2 pi) - log(omega sp/2)/(2 pi)),
//   D_ii = -dt kappa sp/(4 pi).
__global__ void diag_table(const SrcRec* __restrict__ src, double4* __restrict__ diag, int n, double R0, double dt,
                           double omega) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const SrcRec s = src[i];
    const double sp = s.sp;
    diag[i] = double4{R0 * (-sp * kInv4Pi) + dt * sp * (-kEulerGamma - log(0.5 * omega * sp)) * (2.0 * kInv4Pi),
                      0.25 * dt * sp, -dt * s.kappa * sp * kInv4Pi, 0.0};
  }
}

// Source blocks of the single-precision sweep: for each block of 32 sources,
// their positions as 32 FP64 pairs (512 bytes), then 32 FP32 quadruples
// (nx, ny, w/4, 0) (512 bytes).  A step of the sweep loads one block (one
// 16-byte chunk per lane of a wave), and the four lane groups of a wave read
// records 16 bytes apart.  Sources past n repeat the last node with zero
// weight.
__global__ void src_blocks(const SrcRec* __restrict__ src, uint4* blk, int n, int nb) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nb * 32; j += gridDim.x * blockDim.x) {
    const SrcRec s = src[j < n ? j : n - 1];
    double2* xy = reinterpret_cast<double2*>(blk + (size_t)(j / 32) * 64);
    float4* nw = reinterpret_cast<float4*>(blk + (size_t)(j / 32) * 64 + 32);
    xy[j % 32] = make_double2(s.x, s.y);
    nw[j % 32] = make_float4(s.nxf, s.nyf, j < n ? s.wf : 0.0f, 0.0f);
  }
}

int build_diag(dp_problem* p) {
  const int n = (int)p->n;
  DP_TRY(p->diag.reserve((size_t)n * sizeof(double4)));
  diag_table<<<grid1d(n), 256, 0, p->ctx->stream>>>(p->src.as<SrcRec>(), p->diag.as<double4>(), n, p->R0,
                                                    2.0 * kPi / n, p->omega);
  const int nb = (n + 31) / 32;
  DP_TRY(p->srcblk.reserve((size_t)nb * 64 * sizeof(uint4)));
  src_blocks<<<grid1d((size_t)nb * 32), 256, 0, p->ctx->stream>>>(p->src.as<SrcRec>(), p->srcblk.as<uint4>(), n, nb);
  DP_HIP(hipGetLastError());
  return DP_OK;
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
