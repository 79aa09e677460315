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
#include "dp_internal.hpp"

namespace dp {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

struct Tgt {
  double x, y, nx, ny;
};

template <int OP>
struct Nd {
  static constexpr int v = (OP == OP_HARD) ? 2 : 1;
};

// Kernel values of one ordered pair (i, j) from its Hankel values
// (self pairs i == j return 0).
template <int OP>
__device__ __forceinline__ void assemble_pair(const Tgt& t, const SrcRec& s, double dx, double dy, double rinv,
                                              const H01& h, double Ck, bool self, double omega, double eta,
                                              double dt, cplx* K) {
  const double w = dt * s.sp;   // trapezoid weight
  const double ck = Ck * s.sp;  // Kress correction weight
  if constexpr (OP == OP_SOFT) {
    const double nd = (s.nx * dx + s.ny * dy) * rinv;
    // K = (i omega/4) H1 nd + (eta/4) H0,  K1 = -(omega/(4pi)) J1 nd + i eta J0/(4pi)
    const double a = 0.25 * omega * nd, b = 0.25 * eta;
    K[0].re = w * fma(-a, h.h1.im, b * h.h0.re) - ck * (omega * kInv4Pi) * nd * h.h1.re;
    K[0].im = w * fma(a, h.h1.re, b * h.h0.im) + ck * (eta * kInv4Pi) * h.h0.re;
  } else if constexpr (OP == OP_S) {
    K[0].re = -0.25 * w * h.h0.im - ck * kInv4Pi * h.h0.re;
    K[0].im = 0.25 * w * h.h0.re;
  } else if constexpr (OP == OP_D) {
    const double nd = (s.nx * dx + s.ny * dy) * rinv;
    K[0].re = -0.25 * omega * nd * w * h.h1.im - ck * omega * kInv4Pi * nd * h.h1.re;
    K[0].im = 0.25 * omega * nd * w * h.h1.re;
  } else if constexpr (OP == OP_DP) {
    const double ni = (t.nx * dx + t.ny * dy) * rinv;
    K[0].re = 0.25 * omega * ni * w * h.h1.im + ck * omega * kInv4Pi * ni * h.h1.re;
    K[0].im = -0.25 * omega * ni * w * h.h1.re;
  } else {  // OP_HARD
    const double ni = (t.nx * dx + t.ny * dy) * rinv;
    const double Sre = -0.25 * w * h.h0.im - ck * kInv4Pi * h.h0.re;
    const double Sim = 0.25 * w * h.h0.re;
    const double Dre = 0.25 * omega * ni * w * h.h1.im + ck * omega * kInv4Pi * ni * h.h1.re;
    const double Dim = -0.25 * omega * ni * w * h.h1.re;
    const double g = (omega * omega / eta) * (t.nx * s.nx + t.ny * s.ny);
    K[0] = {Sre, Sim};
    // G = -i g S - D'
    K[1] = {g * Sim - Dre, -g * Sre - Dim};
  }
  if (self) {
#pragma unroll
    for (int d = 0; d < Nd<OP>::v; ++d) K[d] = {0.0, 0.0};
  }
}

// Kernel values of one ordered pair (i, j), i != j (self pairs return 0).
template <int OP>
__device__ __forceinline__ void pair_kernel(const Tgt& t, const SrcRec& s, double Ck, bool self,
                                            double omega, double eta, double dt, cplx* K) {
  const double dx = t.x - s.x, dy = t.y - s.y;
  double r2 = fma(dx, dx, dy * dy);
  r2 = self ? 1.0 : r2;
  const double rinv = dp_rsqrt(r2);
  const double r = r2 * rinv;
  const H01 h = hankel01(omega * r);
  assemble_pair<OP>(t, s, dx, dy, rinv, h, Ck, self, omega, eta, dt, K);
}

// Small-argument version (omega r < DP_HANKEL_ZA, the recurrence branch only).
template <int OP>
__device__ __forceinline__ void pair_kernel_near(const Tgt& t, const SrcRec& s, double Ck, double omega, double eta,
                                                 double dt, cplx* K) {
  const double dx = t.x - s.x, dy = t.y - s.y;
  const double r2 = fma(dx, dx, dy * dy);
  const double rinv = dp_rsqrt(r2);
  const H01 h = hankel01_near(omega * r2 * rinv);
  assemble_pair<OP>(t, s, dx, dy, rinv, h, Ck, false, omega, eta, dt, K);
}

// Branch-free version for pairs with omega r >= DP_HANKEL_ZA (asymptotic
// branch only).  `near` reports whether the pair needs the other branch; its
// values are then replaced by pair_kernel.
template <int OP>
__device__ __forceinline__ void pair_kernel_far(const Tgt& t, const SrcRec& s, double Ck, bool self,
                                                double omega, double eta, double dt, cplx* K, bool& near) {
  const double dx = t.x - s.x, dy = t.y - s.y;
  double r2 = fma(dx, dx, dy * dy);
  r2 = self ? 1.0 : r2;
  const double rinv = dp_rsqrt(r2);
  const double z = omega * r2 * rinv;
  near = z < DP_HANKEL_ZA && !self;
  const H01 h = hankel01_far(fmax(z, DP_HANKEL_ZA));
  assemble_pair<OP>(t, s, dx, dy, rinv, h, Ck, self, omega, eta, dt, K);
}

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
    pair_kernel<OP>(t, s, Ck, ii == j, p.omega, p.eta, p.dt, K);
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
        pair_kernel<OP>(t, p.src[j], p.C[k], ii == j, p.omega, p.eta, p.dt, K);
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

// Many-column sweep on the matrix cores.  The contraction
//   out_d[i][c] += sum_j K_d(i, j) dens_d[j][c]
// is a dense complex GEMM whose left operand is generated on the fly: a
// 16 x 4 tile of kernel values (16 targets x 4 sources, one pair per lane)
// is exactly the A operand of v_mfma_f64_16x16x4 (A[i][k] in lane i + 16k),
// and the densities of the same 4 sources for 16 columns are its B operand
// (B[k][c] in lane c + 16k), read straight from the packed density array
// (L2 / MALL resident, coalesced 16-column runs); with no barriers the two
// waves sharing a SIMD drift out of phase.
// Complex products take four real MFMAs (re.re, -im.im into the real
// accumulator; re.im, im.re into the imaginary one); results land in
// D[i][c] = register r of lane c + 16 (i mod 4), i = 4r + lane/16.
// Block: 4 row groups x 16 targets = 64 targets; CH waves per row group split
// the 16*NCBW*CH columns, so each wave keeps only its share of accumulators
// and two waves fit per SIMD: the VALU work of one wave's kernel evaluation
// overlaps the MFMA work of the other (each evaluates its own pairs).
template <int OP, int NCBW>
__global__ __launch_bounds__(512) void sweep_mfma(SweepParams p) {
  constexpr int ND = Nd<OP>::v;
  constexpr int NC = 32 * NCBW;        // columns of the block (two waves per row group)
  __shared__ cplx Kx[2][4][2][ND][64];  // [buffer][row group][step parity][density][lane]
  const int n = p.n;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int rg = wv & 3;                // row group: 16 targets
  const int ch = wv >> 2;               // column half; also the parity of the k-steps it evaluates
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
  // 3-multiplication complex products: T1 += Kr Br, T2 += Ki Bi,
  // T3 += (Kr + Ki)(Br + Bi); then Re = T1 - T2, Im = T3 - T1 - T2.
  dbl4 T1[ND][NCBW], T2[ND][NCBW], T3[ND][NCBW];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int cb = 0; cb < NCBW; ++cb) {
      T1[d][cb] = dbl4{0.0, 0.0, 0.0, 0.0};
      T2[d][cb] = dbl4{0.0, 0.0, 0.0, 0.0};
      T3[d][cb] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  for (int sp = 0; sp < npairs; ++sp) {
    // kernel values of this wave's k-step 2 sp + ch (target i, source j0 + 4 st + lk)
    const int st = 2 * sp + ch;
    const int j = j0 + 4 * st + lk;
    const bool valid = j < j1;
    const int jc = valid ? j : j1 - 1;
    int k = ii - jc;
    k += (k < 0) ? n : 0;
    const SrcRec sr = p.src[jc];
    const double Ck = p.C[k];
    cplx K[ND];
    bool near;
    pair_kernel_far<OP>(t, sr, Ck, ii == jc, p.omega, p.eta, p.dt, K, near);
    if (__builtin_amdgcn_ballot_w64(near)) {
      if (near) pair_kernel_near<OP>(t, sr, Ck, p.omega, p.eta, p.dt, K);
    }
    const int buf = sp & 1;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      K[d] = valid ? K[d] : cplx{0.0, 0.0};
      Kx[buf][rg][ch][d][lane] = K[d];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int sth = 2 * sp + h;
      if (sth >= nsteps) break;
      const int jh = min(j0 + 4 * sth + lk, j1 - 1);
      const cplx* dj = p.dens + (size_t)jh * ND * NC + c0 + li;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const cplx Kh = (h == ch) ? K[d] : Kx[buf][rg][h][d][lane];
        const double ks = Kh.re + Kh.im;
#pragma unroll
        for (int cb = 0; cb < NCBW; ++cb) {
          const cplx B = dj[d * NC + cb * 16];
          T1[d][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Kh.re, B.re, T1[d][cb], 0, 0, 0);
          T2[d][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Kh.im, B.im, T2[d][cb], 0, 0, 0);
          T3[d][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ks, B.re + B.im, T3[d][cb], 0, 0, 0);
        }
      }
    }
  }
  const int rbase = blockIdx.x * 64 + rg * 16;
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int cb = 0; cb < NCBW; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rbase + 4 * r + lk;
        if (row < n) {
          const double t1 = T1[d][cb][r], t2 = T2[d][cb][r], t3 = T3[d][cb][r];
          p.partial[(((size_t)blockIdx.y * ND + d) * NC + c0 + cb * 16 + li) * n + row] =
              cplx{t1 - t2, t3 - t1 - t2};
        }
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

struct EpiParams {
  const SrcRec* src;
  const cplx* partial;
  const cplx* q;       // density (n x nrhs), for diagonal and identity terms
  const cplx* q2;      // second density (hard: sigma1) or null
  cplx* out0;          // result (soft/layer) or u (hard)
  cplx* out1;          // v (hard)
  int n, nrhs, nrp, nchunks, op, col0;
  double omega, eta, dt, R0;
};

// Sum chunk partials, add the diagonal (Kress limits) and identity terms.
__global__ void sweep_epilogue(EpiParams e) {
  const size_t tot = (size_t)e.n * e.nrhs;
  const int nd = e.op == OP_HARD ? 2 : 1;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = idx % e.n;
    const int c = idx / e.n;
    const SrcRec s = e.src[i];
    const double sp = s.sp;
    // S_ii = R0 (-sp/(4 pi)) + dt sp (i/4 - gamma/(2 pi) - log(omega sp/2)/(2 pi))
    const cplx Sii = {e.R0 * (-sp * kInv4Pi) +
                          e.dt * sp * (-kEulerGamma - log(0.5 * e.omega * sp)) * (2.0 * kInv4Pi),
                      0.25 * e.dt * sp};
    const double Dii = -e.dt * s.kappa * sp * kInv4Pi;  // D_ii = D'_ii
    cplx sum[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int ch = 0; ch < e.nchunks; ++ch)
      for (int d = 0; d < nd; ++d) {
        const cplx v = e.partial[(((size_t)ch * nd + d) * e.nrp + c) * e.n + i];
        sum[d].re += v.re;
        sum[d].im += v.im;
      }
    const cplx qi = e.q[(size_t)(e.col0 + c) * e.n + i];
    const size_t o = (size_t)(e.col0 + c) * e.n + i;
    if (e.op == OP_SOFT) {
      // (1/2 + D_ii - i eta S_ii) q_i
      const cplx a = {0.5 + Dii + e.eta * Sii.im, -e.eta * Sii.re};
      cfma(sum[0], a, qi);
      e.out0[o] = sum[0];
    } else if (e.op == OP_S) {
      cfma(sum[0], Sii, qi);
      e.out0[o] = sum[0];
    } else if (e.op == OP_D || e.op == OP_DP) {
      cfma(sum[0], cplx{Dii, 0.0}, qi);
      e.out0[o] = sum[0];
    } else {
      const cplx s1 = e.q2[(size_t)(e.col0 + c) * e.n + i];
      cfma(sum[0], Sii, s1);
      // G_ii = -i (omega^2/eta) S_ii - D'_ii
      const double g = e.omega * e.omega / e.eta;
      cfma(sum[1], cplx{g * Sii.im - Dii, -g * Sii.re}, qi);
      e.out0[o] = sum[0];
      e.out1[o] = sum[1];
    }
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
      case 32: sweep_mfma<OP, 1><<<grid, 512, 0, st>>>(sp); break;
      default: sweep_mfma<OP, 2><<<grid, 512, 0, st>>>(sp); break;
    }
  }
}

static int pad_cols(int nrhs) {
  int r = 1;
  while (r < nrhs && r < 64) r *= 2;
  return r;
}

// Core sweep over one group of <= 64 columns.  a (and b for hard) are the
// densities; results go to out0 (and out1).
static int sweep_group(dp_problem* p, int op, int nrhs, int col0, const cplx* a, const cplx* b,
                       cplx* out0, cplx* out1) {
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n;
  const int nd = op == OP_HARD ? 2 : 1;
  const int nrp = pad_cols(nrhs);
  const int rows_per_block = nrp <= 4 ? 256 : 64;
  const int bx = (n + rows_per_block - 1) / rows_per_block;
  int nchunks = (2048 + bx - 1) / bx;
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
    pack_dens<<<grid1d(tot), 256, 0, st>>>(a, b, p->dens.as<cplx>(), n, nrhs, nrp, nd, col0);
  }
  SweepParams sp;
  sp.src = p->src.as<SrcRec>();
  sp.C = p->C.as<double>();
  sp.dens = p->dens.as<cplx>();
  sp.partial = p->partial.as<cplx>();
  sp.n = n;
  sp.nrp = nrp;
  sp.nd = nd;
  sp.chunk_len = chunk_len;
  sp.nchunks = nchunks;
  sp.omega = p->omega;
  sp.eta = p->eta;
  sp.dt = 2.0 * kPi / n;
  p->clock.start(st);
  switch (op) {
    case OP_SOFT: launch_sweep<OP_SOFT>(sp, nrp, st); break;
    case OP_HARD: launch_sweep<OP_HARD>(sp, nrp, st); break;
    case OP_S: launch_sweep<OP_S>(sp, nrp, st); break;
    case OP_D: launch_sweep<OP_D>(sp, nrp, st); break;
    default: launch_sweep<OP_DP>(sp, nrp, st); break;
  }
  p->clock.stop(st);
  DP_HIP(hipGetLastError());
  EpiParams e;
  e.src = sp.src;
  e.partial = sp.partial;
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
  sweep_epilogue<<<grid1d((size_t)n * nrhs), 256, 0, st>>>(e);
  DP_HIP(hipGetLastError());
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

int sweep_apply(dp_problem* p, int op, int nrhs, const cplx* q, cplx* y) {
  for (int c0 = 0; c0 < nrhs; c0 += 64) {
    const int nc = nrhs - c0 < 64 ? nrhs - c0 : 64;
    DP_TRY(sweep_group(p, op, nc, c0, q, nullptr, y, nullptr));
  }
  return DP_OK;
}

int matvec(dp_problem* p, int nrhs, const cplx* q, cplx* y) {
  if (p->kind == DP_SOFT) return sweep_apply(p, OP_SOFT, nrhs, q, y);
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
    DP_TRY(sweep_group(p, OP_HARD, nc, c0, sig, q, u, v));
  }
  DP_TRY(spectral_derivative(p, nrhs, u, sig));
  hard_combine<<<grid1d(tot), 256, 0, p->ctx->stream>>>(q, v, sig, y, tot, p->eta);
  DP_HIP(hipGetLastError());
  return DP_OK;
}

}  // namespace dp
