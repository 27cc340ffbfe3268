// taps.hpp — the depth-dependent pencil-beam kernel of one beam-frame plane
// (arXiv:2512.18863 §2.2.5).
//
// Radially symmetric double-exponential kernel with unit plane integral,
//   p(r; z) = (A e^{-a r} + B e^{-b r}) / (2 pi r (A/a + B/b)),
// whose parameters A, a, B, b are cubics in the central-axis water-equivalent
// depth z of the plane (clamped to [0, kz_max]).  Taps sit on the plane's own
// grid, spacing delta = Delta d_k / SAD:
//   K[p][q] = delta^2 p(delta sqrt(p^2 + q^2); z)   off centre,
//   K[0][0] = integral of p over the disc of area delta^2.
// The truncated kernel is not renormalised (what lies beyond the n x n window is
// the kernel-size effect the paper studies).
#pragma once

#include "device_math.hpp"

namespace pdrt {

template <typename T>
struct TapParams {
  T A, a, B, b, Aa, Bb, inv_norm, delta;
};

template <typename T>
__device__ __forceinline__ TapParams<T> tap_params(const Geo<T>& g, int k, T zk) {
  TapParams<T> t;
  T z = fmin(fmax(zk, T(0)), g.kz_max);
  t.A = g.kpoly[0][0] + z * (g.kpoly[0][1] + z * (g.kpoly[0][2] + z * g.kpoly[0][3]));
  t.a = g.kpoly[1][0] + z * (g.kpoly[1][1] + z * (g.kpoly[1][2] + z * g.kpoly[1][3]));
  t.B = g.kpoly[2][0] + z * (g.kpoly[2][1] + z * (g.kpoly[2][2] + z * g.kpoly[2][3]));
  t.b = g.kpoly[3][0] + z * (g.kpoly[3][1] + z * (g.kpoly[3][2] + z * g.kpoly[3][3]));
  t.Aa = t.A / t.a;
  t.Bb = t.B / t.b;
  t.inv_norm = T(1) / (t.Aa + t.Bb);
  t.delta = g.lat * (T(1) + (g.e0 + T(k) * g.dstep) * g.inv_sad);
  return t;
}

template <typename T>
__device__ __forceinline__ T tap_value(const TapParams<T>& t, int p, int q) {
  const T two_pi = T(6.283185307179586476925286766559);
  const T inv_sqrt_pi = T(0.56418958354775628694807945156077);
  if (p == 0 && q == 0) {
    T r0 = t.delta * inv_sqrt_pi;
    return (t.Aa * -expm1(-t.a * r0) + t.Bb * -expm1(-t.b * r0)) * t.inv_norm;
  }
  T rr = t.delta * dsqrt(T(p * p + q * q));
  return t.delta * t.delta * (t.A * dexp(-t.a * rr) + t.B * dexp(-t.b * rr)) * t.inv_norm / (two_pi * rr);
}

}  // namespace pdrt
