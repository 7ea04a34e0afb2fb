// fm_steer.h -- steering-vector phasors shared by the spectrum passes
// (a_m(theta) = exp(-j pi m sin(theta)), eq. (5)); device code only.
#pragma once

#include "fm_internal.h"

namespace fm {
namespace steer {

constexpr double kTwo64 = 18446744073709551616.0;

// F = frac(-sin(theta)/2) * 2^64: turns per element as a 64-bit fraction
__device__ inline unsigned long long turn_freq(double theta0, double dtheta, int l) {
  const double th = fma((double)l, dtheta, theta0);
  const double s = sin(th * (3.141592653589793 / 180.0));
  double f = -0.5 * s;
  f = f - floor(f);
  double x = f * kTwo64;
  if (!(x < kTwo64)) x = 0.0;
  return (unsigned long long)x;
}

// exp(2 pi j * (m F mod 2^64) / 2^64) in FP32 from the top 32 phase bits
__device__ inline float2 phasor32(unsigned m, unsigned long long F, const float2 *tab) {
  const unsigned lo = (unsigned)F, hi = (unsigned)(F >> 32);
  const unsigned top = m * hi + __umulhi(m, lo);
  const float d = (float)(top & 0xFFFFFFu) * 1.4629180792671596e-09f;  // 2 pi / 2^32
  const float d2 = d * d;
  const float c = fmaf(d2, fmaf(d2, 1.0f / 24.0f, -0.5f), 1.0f);
  const float s = d * fmaf(d2, fmaf(d2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
  const float2 t = tab[top >> 24];
  // explicit fused forms: every kernel variant rounds a phasor identically
  return make_float2(fmaf(t.x, c, -(t.y * s)), fmaf(t.x, s, t.y * c));
}

// the same phasor in FP64
__device__ inline double2 phasor64(unsigned long long m, unsigned long long F) {
  const unsigned long long ph = m * F;
  const double x = (double)(ph >> 11) * 0x1p-52;  // 2 * ph / 2^64, in [0, 2)
  double s, c;
  sincospi(x, &s, &c);
  return make_double2(c, s);
}

// complex product with explicit fused forms (no contraction left to the
// compiler, so the rounding does not depend on the surrounding code)
__device__ inline float2 cmulf(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

}  // namespace steer
}  // namespace fm
