// Device/host math for the CFIE kernels: sin/cos with Cody-Waite reduction
// and the Hankel functions H_0^(1), H_1^(1) of a real positive argument.
//
// The Green's function of the Helmholtz equation is (i/4) H_0^(1)(omega r)
// (Sec. 1); its normal derivatives bring in H_1^(1).  Both are evaluated
// here from published formulas:
//   * z >= DP_HANKEL_ZA: Hankel's asymptotic expansion (DLMF 10.17.5),
//       H_nu(z) ~ sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} sum_k i^k a_k(nu) z^-k,
//       a_k(nu) = prod_{m=1..k} (4 nu^2 - (2m-1)^2) / (k! 8^k),
//     whose even and odd parts P_nu, Q_nu are polynomials in u = 1/z^2,
//     economized on [0, 1/DP_HANKEL_ZA^2] (hankel_poly.hpp, error < 1e-17);
//   * z < DP_HANKEL_ZA: J_0, J_1 by Miller's backward recurrence
//     J_{k-1} = (2k/z) J_k - J_{k+1} normalised by J_0 + 2 sum J_{2k} = 1
//     (DLMF 10.74(iv), 10.12.4), Y_0 by Neumann's expansion in the J_{2k}
//     (Y_0 = (2/pi)[(ln(z/2)+gamma) J_0 - 2 sum_{k>=1} (-1)^k J_{2k}/k]) and
//     Y_1 = -Y_0' from the same series differentiated term by term,
//       Y_1 = (2/pi)[-J_0/z + (ln(z/2)+gamma) J_1 - J_1
//              + sum_{m>=1} (-1)^{m+1} (2m+1)/(m(m+1)) J_{2m+1}].
// sin/cos: x = k pi/2 + r, |r| <= pi/4, with pi/2 split in two doubles and
// fused multiply-adds, then the Taylor series of sin and cos in r economized
// on the reduced range (hankel_poly.hpp).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "hankel_poly.hpp"

#define DP_HD __host__ __device__ __forceinline__

namespace dp {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;
// pi/2 = kPio2Hi + kPio2Lo; kPio2Hi is the double nearest to pi/2 and kPio2Lo
// the double nearest to the remainder (pi/2 evaluated to 40 digits).
constexpr double kPio2Hi = 1.5707963267948966192313216916397514;
constexpr double kPio2Lo = 6.123233995736766035868820147291819e-17;
constexpr double kTwoOverPi = 0.63661977236758134307553505349005745;
constexpr double kSqrt2OverPi = 0.79788456080286535587989211986876373;
constexpr double kInvSqrt2 = 0.70710678118654752440084436210484904;

struct cplx {
  double re, im;
};

DP_HD cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
DP_HD cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
DP_HD cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
// acc += a * b
DP_HD void cfma(cplx& acc, cplx a, cplx b) {
  acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}

// --------------------------------------------------------------- sin / cos
// Horner evaluation of sum_k c[k] x^k.
template <class T, int N>
DP_HD T horner(const T (&c)[N], T x) {
  T p = c[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) p = fma(p, x, c[k]);
  return p;
}

// sin r = r + r v S(v), cos r = 1 + v C(v), v = r^2, |r| <= pi/4.
DP_HD void sincos_reduced(double r, double& s, double& c) {
  const double v = r * r;
  s = fma(r * v, horner(kSinS, v), r);
  c = fma(v, horner(kCosC, v), 1.0);
}

// sin and cos of x for |x| < 2^40.
DP_HD void dp_sincos(double x, double& s, double& c) {
  const double k = rint(x * kTwoOverPi);
  double r = fma(-k, kPio2Hi, x);
  r = fma(-k, kPio2Lo, r);
  double sr, cr;
  sincos_reduced(r, sr, cr);
  const long long q = (long long)k & 3;
  // x = k pi/2 + r: rotate (cos r, sin r) by q quarter turns
  const double s1 = (q & 1) ? cr : sr;
  const double c1 = (q & 1) ? sr : cr;
  s = (q & 2) ? -s1 : s1;
  c = ((q + 1) & 2) ? -c1 : c1;
}

DP_HD double dp_rsqrt(double z) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __ocml_rsqrt_f64(z);
#else
  return 1.0 / sqrt(z);
#endif
}

// --------------------------------------------------------------- Hankel
constexpr double DP_HANKEL_ZA = kHankelZA;  // branch point; the far polynomials are fitted above it

struct H01 {
  cplx h0, h1;
};

// Asymptotic branch, z >= DP_HANKEL_ZA: H_nu = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)}
// (P_nu + i Q_nu), P_nu and Q_nu/t polynomials in u = t^2, t = 1/z.
DP_HD H01 hankel01_far(double z) {
  const double y = dp_rsqrt(z);
  const double t = y * y;
  const double u = t * t;
  const double p0 = horner(kHankP0, u), p1 = horner(kHankP1, u);
  const double q0 = horner(kHankQ0, u) * t, q1 = horner(kHankQ1, u) * t;
  double s, c;
  dp_sincos(z, s, c);
  const double m = kSqrt2OverPi * y * kInvSqrt2;
  // e^{i(z - pi/4)} = ((c + s) + i (s - c))/sqrt2 ; e^{i(z - 3pi/4)} = ((s - c) - i (s + c))/sqrt2
  const cplx e0 = {(c + s) * m, (s - c) * m};
  const cplx e1 = {(s - c) * m, -(s + c) * m};
  H01 h;
  h.h0 = cmul(e0, cplx{p0, q0});
  h.h1 = cmul(e1, cplx{p1, q1});
  return h;
}

// Small/moderate argument branch, 0 < z < DP_HANKEL_ZA.
DP_HD H01 hankel01_near(double z) {
  const int N = 2 * (int)((z + 41.0) * 0.5);  // even start index, J_N(z) < 1e-19 J_0
  const double tz = 2.0 / z;
  double jp1 = 0.0, jk = 1e-30;  // J_{k+1}, J_k (unnormalised), k = N
  double norm = 0.0, s0 = 0.0, s1 = 0.0;
  for (int k = N; k >= 1; --k) {
    const double jm1 = fma((double)k * tz, jk, -jp1);  // J_{k-1}
    const int idx = k - 1;
    if (idx >= 2 && !(idx & 1)) {
      const int m = idx >> 1;
      norm = fma(2.0, jm1, norm);
      s0 += ((m & 1) ? 1.0 : -1.0) * jm1 / (double)m;  // (-1)^{m+1} J_{2m}/m
    } else if (idx >= 3) {
      const int m = (idx - 1) >> 1;
      s1 += ((m & 1) ? 1.0 : -1.0) * (2.0 * m + 1.0) / ((double)m * (m + 1.0)) * jm1;
    }
    jp1 = jk;
    jk = jm1;
    if (fabs(jk) > 1e250) {
      jp1 *= 1e-250;
      jk *= 1e-250;
      norm *= 1e-250;
      s0 *= 1e-250;
      s1 *= 1e-250;
    }
  }
  // now jk = J_0, jp1 = J_1 (unnormalised)
  norm += jk;
  const double sc = 1.0 / norm;
  const double J0 = jk * sc, J1 = jp1 * sc;
  s0 *= sc;
  s1 *= sc;
  const double lg = log(0.5 * z) + kEulerGamma;
  const double Y0 = (2.0 / kPi) * (lg * J0 + 2.0 * s0);
  const double Y1 = (2.0 / kPi) * (-J0 / z + lg * J1 - J1 + s1);
  H01 h;
  h.h0 = {J0, Y0};
  h.h1 = {J1, Y1};
  return h;
}

DP_HD H01 hankel01(double z) { return z >= DP_HANKEL_ZA ? hankel01_far(z) : hankel01_near(z); }

// ----------------------------------------------------- single precision
struct cplxf {
  float re, im;
};

struct H01f {
  cplxf h0, h1;
};

DP_HD float dp_rsqrtf(float z) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(z);
#else
  return 1.0f / sqrtf(z);
#endif
}

// Asymptotic branch for z >= DP_HANKEL_ZA with FP32 arithmetic, with the
// argument in quarter turns, w = 2 z / pi (FP64).  The reduction
// f = w - rint(w), |f| <= 1/2, is exact in FP64 (|w| up to 1e6 keeps ~1e-16
// absolute phase error); everything after it is FP32 with the quarter-turn
// polynomials of hankel_poly.hpp (sine and cosine of (pi/2) f to ~5e-8, the
// amplitude polynomials in s = 1/w^2 to ~4e-9).  Relative accuracy ~3e-7.
// Both values come out multiplied by `scale` (a power of two, or 1, and
// never negative).
// With z = (pi/2)(q + f), e^{i(z - pi/4)} sqrt(2) = (c + s) + i (s - c) for
// c = cos z, s = sin z; in terms of P = cos + sin and M = cos - sin of
// (pi/2) f that pair is (P, -M), (M, P), (-P, M), (-M, -P) for
// q = 0, 1, 2, 3 mod 4.  The amplitude sqrt(2/(pi z)) is (2/pi)/sqrt(w);
// its constant (2/pi)/sqrt(2) (with the 1/sqrt(2) of P and M) is folded into
// the sine and cosine polynomials, and the sign of q = 2, 3 is set on the
// non-negative magnitude as its sign bit.
DP_HD H01f hankel01_far32w(double w, float scale = 1.0f) {
  const double kq = rint(w);
  const float fr = (float)(w - kq), v = fr * fr;
  const float sr = fr * horner(kSinQ32, v);  // kappa sin((pi/2) f)
  const float cr = horner(kCosQ32, v);       // kappa cos((pi/2) f)
  const int q = (int)kq;  // kq < 2^31 for w < 2e9
  const float P = cr + sr, M = cr - sr;
  const float a = (q & 1) ? M : P;
  const float b = (q & 1) ? P : -M;
  const float y = dp_rsqrtf((float)w);  // 1/sqrt(w)
  const float tw = y * y;                // 1/w
  const float s = tw * tw;
  const float p0 = horner(kHankP0W32, s), p1 = horner(kHankP1W32, s);
  const float q0 = horner(kHankQ0W32, s) * tw, q1 = horner(kHankQ1W32, s) * tw;
  const float m0 = scale * y;
  const float m = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, m0) | ((uint32_t)(q & 2) << 30));
  const cplxf e0 = {a * m, b * m};  // e1 = -i e0
  H01f h;
  h.h0 = {e0.re * p0 - e0.im * q0, e0.re * q0 + e0.im * p0};
  h.h1 = {e0.im * p1 + e0.re * q1, e0.im * q1 - e0.re * p1};
  return h;
}

}  // namespace dp
