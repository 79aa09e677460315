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
// phase is reduced modulo pi/2 in FP64 inside hankel01_far32), everything
// after the reduction is FP32.  Near-field pairs are left to the FP64
// near-field pass, as in the FP64 sweep.
template <int OP>
struct Nd32 {
  static constexpr int v = Nd<OP>::v;
};

// Kernel values of one pair from FP32 Hankel values; the source's normal,
// trapezoid weight and speed come from its FP32 copies.
template <int OP>
__device__ __forceinline__ void assemble_pair32(const Tgt& t, const SrcRec& s, float dx, float dy, float rinv,
                                                const H01f& h, float Ck, bool self, float omega, float eta,
                                                cplxf* K) {
  constexpr float k4 = (float)kInv4Pi;
  const float w = s.wf;
  const float ck = Ck * s.spf;
  if constexpr (OP == OP_SOFT) {
    const float nd = (s.nxf * dx + s.nyf * dy) * rinv;
    const float a = 0.25f * omega * nd, b = 0.25f * eta;
    K[0].re = w * fmaf(-a, h.h1.im, b * h.h0.re) - ck * (omega * k4) * nd * h.h1.re;
    K[0].im = w * fmaf(a, h.h1.re, b * h.h0.im) + ck * (eta * k4) * h.h0.re;
  } else if constexpr (OP == OP_S) {
    K[0].re = -0.25f * w * h.h0.im - ck * k4 * h.h0.re;
    K[0].im = 0.25f * w * h.h0.re;
  } else if constexpr (OP == OP_D) {
    const float nd = (s.nxf * dx + s.nyf * dy) * rinv;
    K[0].re = -0.25f * omega * nd * w * h.h1.im - ck * omega * k4 * nd * h.h1.re;
    K[0].im = 0.25f * omega * nd * w * h.h1.re;
  } else if constexpr (OP == OP_DP) {
    const float ni = ((float)t.nx * dx + (float)t.ny * dy) * rinv;
    K[0].re = 0.25f * omega * ni * w * h.h1.im + ck * omega * k4 * ni * h.h1.re;
    K[0].im = -0.25f * omega * ni * w * h.h1.re;
  } else {
    const float ni = ((float)t.nx * dx + (float)t.ny * dy) * rinv;
    const float Sre = -0.25f * w * h.h0.im - ck * k4 * h.h0.re;
    const float Sim = 0.25f * w * h.h0.re;
    const float Dre = 0.25f * omega * ni * w * h.h1.im + ck * omega * k4 * ni * h.h1.re;
    const float Dim = -0.25f * omega * ni * w * h.h1.re;
    const float g = (omega * omega / eta) * ((float)t.nx * s.nxf + (float)t.ny * s.nyf);
    K[0] = {Sre, Sim};
    K[1] = {g * Sim - Dre, -g * Sre - Dim};
  }
  if (self) {
#pragma unroll
    for (int d = 0; d < Nd<OP>::v; ++d) K[d] = {0.0f, 0.0f};
  }
}

// Far-field pair with FP32 kernel values.  1/r comes from the FP32 reciprocal
// square root refined by one Newton step in FP64 (relative error ~2e-14), so
// the phase omega r keeps an absolute error below 1e-9 for omega r < 5e4.
template <int OP>
__device__ __forceinline__ void pair_kernel_far32(const Tgt& t, const SrcRec& s, double Ck, bool self, double omega,
                                                  double eta, double r2near, cplxf* K) {
  const double dx = t.x - s.x, dy = t.y - s.y;
  double r2 = pair_r2(t.x, t.y, s.x, s.y);
  const bool zero = self || r2 < r2near;
  r2 = self ? 1.0 : r2;
  const double y0 = (double)dp_rsqrtf((float)r2);
  const double rinv = y0 * fma(-0.5 * r2, y0 * y0, 1.5);
  const double z = omega * (r2 * rinv);
  const H01f h = hankel01_far32(fmax(z, DP_HANKEL_ZA));
  assemble_pair32<OP>(t, s, (float)dx, (float)dy, (float)rinv, h, (float)Ck, zero, (float)omega, (float)eta, K);
}

// ------------------------------------------------------------ epilogue
struct EpiParams {
  const SrcRec* src;
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
// diagonal (Kress limits) and the identity terms, in FP64.
template <class PT>
__global__ void sweep_epilogue(EpiParams e) {
  const size_t tot = (size_t)e.n * e.nrhs;
  const int nd = e.op == OP_HARD ? 2 : 1;
  const PT* part = static_cast<const PT*>(e.partial);
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
    if (e.nearp)
      for (int d = 0; d < nd; ++d) sum[d] = e.nearp[((size_t)d * e.nrp + c) * e.n + i];
    for (int ch = 0; ch < e.nchunks; ++ch)
      for (int d = 0; d < nd; ++d) {
        const PT v = part[(((size_t)ch * nd + d) * e.nrp + c) * e.n + i];
        sum[d].re += (double)v.re;
        sum[d].im += (double)v.im;
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
