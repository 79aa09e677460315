// Per-pair kernel values of the sweep (device code shared by the FP64 and
// mixed-precision sweeps).  See sweep.hip for the operators.
#pragma once

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

// Squared distance of a pair.  The near-field list and every sweep evaluate
// it with this one expression, so the two agree on which pairs are near.
__device__ __forceinline__ double pair_r2(double tx, double ty, double sx, double sy) {
  const double dx = tx - sx, dy = ty - sy;
  return fma(dx, dx, dy * dy);
}

// Near-field pair (r^2 < r2near, so omega r is below the asymptotic range):
// small-argument Hankel branch.
template <int OP>
__device__ __forceinline__ void pair_kernel_near(const Tgt& t, const SrcRec& s, double Ck, double omega, double eta,
                                                 double dt, cplx* K) {
  const double dx = t.x - s.x, dy = t.y - s.y;
  const double r2 = pair_r2(t.x, t.y, s.x, s.y);
  const double rinv = dp_rsqrt(r2);
  const H01 h = hankel01_near(omega * r2 * rinv);
  assemble_pair<OP>(t, s, dx, dy, rinv, h, Ck, false, omega, eta, dt, K);
}

// Far-field pair (asymptotic branch only, branch-free).  Self pairs and
// near-field pairs (r^2 < r2near) return 0: the diagonal is added by the
// epilogue and the near field by its own pass.
template <int OP>
__device__ __forceinline__ void pair_kernel_far(const Tgt& t, const SrcRec& s, double Ck, bool self,
                                                double omega, double eta, double dt, double r2near, cplx* K) {
  const double dx = t.x - s.x, dy = t.y - s.y;
  double r2 = pair_r2(t.x, t.y, s.x, s.y);
  const bool zero = self || r2 < r2near;
  r2 = self ? 1.0 : r2;
  const double rinv = dp_rsqrt(r2);
  const double z = omega * r2 * rinv;
  const H01 h = hankel01_far(fmax(z, DP_HANKEL_ZA));
  assemble_pair<OP>(t, s, dx, dy, rinv, h, Ck, zero, omega, eta, dt, K);
}


// ------------------------------------------------------------ mixed precision
// FP32 kernel values: the geometry, r and the phase omega r are FP64 (the
// phase, in quarter turns, is reduced in FP64 inside hankel01_far32w),
// everything after the reduction is FP32.  Near-field pairs are left to the FP64
// near-field pass, as in the FP64 sweep.
template <int OP>
struct Nd32 {
  static constexpr int v = Nd<OP>::v;
};

// Per-launch constants of the FP32 kernel values.  Output scales sc[d] are
// powers of two (1 when unscaled): sc0 multiplies the Hankel values, and the
// hard operator's second density takes the ratio sc1/sc0 in its factors.
struct Far32 {
  double r2near;
  double qt, qh;  // 2 omega / pi (quarter turns of phase per unit distance), omega / pi
  float sc0;   // scale of density 0 (applied to H0, H1)
  float om;    // omega
  float eta;   // eta
  float om_r;  // omega sc1/sc0 (hard)
  float g_r;   // (omega^2/eta) sc1/sc0 (hard)
};

__host__ __device__ inline Far32 far32_consts(double omega, double eta, double r2near, float sc0, float sc1) {
  Far32 f;
  f.r2near = r2near;
  f.qt = 2.0 * omega / kPi;
  f.qh = omega / kPi;
  f.sc0 = sc0;
  f.om = (float)omega;
  f.eta = (float)eta;
  f.om_r = (float)(omega * (double)sc1 / (double)sc0);
  f.g_r = (float)(omega * omega / eta * (double)sc1 / (double)sc0);
  return f;
}

// Target factors of the FP32 kernel values, once per target: its normal
// times the D'-type factor (omega, or omega sc1/sc0 for the hard operator)
// and times (omega^2/eta) sc1/sc0 (hard).
struct Tgt32 {
  float nxo, nyo, nxg, nyg;
};

template <int OP>
__host__ __device__ inline Tgt32 tgt32(double nx, double ny, const Far32& f) {
  const float o = OP == OP_HARD ? f.om_r : f.om;
  return Tgt32{(float)nx * o, (float)ny * o, (float)nx * f.g_r, (float)ny * f.g_r};
}

// max(a, b) for finite a and b as one instruction (fmax first quiets a
// possible signaling NaN in a separate instruction).
__device__ __forceinline__ double max_f64(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Far-field pair with FP32 kernel values.  r comes from the FP32 reciprocal
// square root y0 refined by one Newton step for sqrt in FP64 (relative error
// ~1e-14), computed directly in quarter turns, w = (2 omega / pi) r, so the
// phase keeps an absolute error below 1e-9 for omega r < 5e4; 1/r in the
// FP32 factors is y0 itself.  The source's FP32
// weight wf = dt |x'_j| / 4 multiplies the Hankel values (h = wf H), and
// rho = C_k / (pi dt) is the ratio of the Kress weight C_k |x'_j| / (4 pi) to
// it, so the S-type and D-type values share
//   A0 = Im h0 + rho Re h0,  B1 = Im h1 + rho Re h1
// (S = -A0 + i Re h0, D' = omega nu_i.rhat (B1 - i Re h1)).  Pairs with zero
// set (outside the caller's range) or in the near field (self pairs
// included: r = 0) get wf = 0 and hence K = 0; their squared distance is
// raised to at least r2near, which keeps every value finite and the argument
// of the asymptotic branch at or above DP_HANKEL_ZA.
// The source enters as its position (sx, sy) and the FP32 normal and weight.
template <int OP>
__device__ __forceinline__ void pair_kernel_far32v(const Tgt& t, const Tgt32& tf, double sx, double sy, float snx,
                                                   float sny, float swf, float rho, bool zero, const Far32& f,
                                                   cplxf* K) {
  const double dx = t.x - sx, dy = t.y - sy;
  const double r2p = pair_r2(t.x, t.y, sx, sy);
  zero = zero || r2p < f.r2near;
  const double r2 = max_f64(r2p, f.r2near);
  const float y0 = dp_rsqrtf((float)r2);
  const double yd = (double)y0;
  const double r0 = r2 * yd;
  const double w = fma(yd * f.qh, fma(-r0, r0, r2), r0 * f.qt);  // (2 omega / pi) r
  const float wq = zero ? 0.0f : swf;
  const H01f h = hankel01_far32w(w, f.sc0 * wq);
  const float dxf = (float)dx, dyf = (float)dy;
  const float A0 = fmaf(rho, h.h0.re, h.h0.im);
  const float Sr = h.h0.re;
  if constexpr (OP == OP_S) {
    K[0] = {-A0, Sr};
    return;
  }
  const float B1 = fmaf(rho, h.h1.re, h.h1.im);
  const float T1 = h.h1.re;
  if constexpr (OP == OP_SOFT || OP == OP_D) {
    const float on = fmaf(snx, dxf, sny * dyf) * (y0 * f.om);  // omega nu_j.rhat
    if constexpr (OP == OP_SOFT) K[0] = {fmaf(f.eta, Sr, -on * B1), fmaf(f.eta, A0, on * T1)};
    else K[0] = {-on * B1, on * T1};
  } else if constexpr (OP == OP_DP) {
    const float on = fmaf(tf.nxo, dxf, tf.nyo * dyf) * y0;           // omega nu_i.rhat
    K[0] = {on * B1, -on * T1};
  } else {  // OP_HARD: S and G = -i (omega^2/eta)(nu_i.nu_j) S - D'
    const float on = fmaf(tf.nxo, dxf, tf.nyo * dyf) * y0;           // omega nu_i.rhat sc1/sc0
    const float g = fmaf(tf.nxg, snx, tf.nyg * sny);                  // (omega^2/eta) nu_i.nu_j sc1/sc0
    K[0] = {-A0, Sr};
    K[1] = {fmaf(g, Sr, -on * B1), fmaf(g, A0, on * T1)};
  }
}

template <int OP>
__device__ __forceinline__ void pair_kernel_far32(const Tgt& t, const Tgt32& tf, const SrcRec& s, float rho,
                                                  bool zero, const Far32& f, cplxf* K) {
  pair_kernel_far32v<OP>(t, tf, s.x, s.y, s.nxf, s.nyf, s.wf, rho, zero, f, K);
}

// ------------------------------------------------------------ epilogue
struct EpiParams {
  const SrcRec* src;
  const double4* diag;  // per node: S_ii (re, im), D_ii
  const void* partial;
  const cplx* nearp;   // near-field sums [nd][nrp][n] (FP64) or null
  const cplx* q;       // density (n x nrhs), for diagonal and identity terms
  const cplx* q2;      // second density (hard: sigma1) or null
  cplx* out0;          // result (soft/layer) or u (hard)
  cplx* out1;          // v (hard)
  int n, nrhs, nrp, nchunks, op, col0;
  double omega, eta, dt, R0;
};

// Sum the near-field sums and the chunk partials (FP64 or FP32), add the
// diagonal (Kress limits, per-row table) and the identity terms, in FP64.
// The partials of four chunks are requested together.
template <class PT>
__global__ void sweep_epilogue(EpiParams e) {
  const size_t tot = (size_t)e.n * e.nrhs;
  const int nd = e.op == OP_HARD ? 2 : 1;
  const PT* part = static_cast<const PT*>(e.partial);
  const size_t cs = (size_t)nd * e.nrp * e.n;  // elements between chunks
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = idx % e.n;
    const int c = idx / e.n;
    const double4 dg = e.diag[i];  // S_ii (re, im), D_ii = D'_ii
    const cplx Sii = {dg.x, dg.y};
    const double Dii = dg.z;
    cplx sum[2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (e.nearp)
      for (int d = 0; d < nd; ++d) sum[d] = e.nearp[((size_t)d * e.nrp + c) * e.n + i];
    for (int d = 0; d < nd; ++d) {
      const PT* pd = part + ((size_t)d * e.nrp + c) * e.n + i;
      int ch = 0;
      for (; ch + 4 <= e.nchunks; ch += 4) {
        PT v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = pd[(ch + u) * cs];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          sum[d].re += (double)v[u].re;
          sum[d].im += (double)v[u].im;
        }
      }
      for (; ch < e.nchunks; ++ch) {
        const PT v = pd[ch * cs];
        sum[d].re += (double)v.re;
        sum[d].im += (double)v.im;
      }
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

}  // namespace dp
