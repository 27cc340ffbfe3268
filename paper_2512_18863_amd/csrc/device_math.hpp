// device_math.hpp — small device helpers shared by the dose kernels.
#pragma once

#include "pdrt_internal.hpp"

namespace pdrt {

template <typename T>
__device__ __forceinline__ T dfloor(T x);
template <>
__device__ __forceinline__ float dfloor<float>(float x) { return floorf(x); }
template <>
__device__ __forceinline__ double dfloor<double>(double x) { return floor(x); }

template <typename T>
__device__ __forceinline__ T dexp(T x);
template <>
__device__ __forceinline__ float dexp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double dexp<double>(double x) { return exp(x); }

template <typename T>
__device__ __forceinline__ T dsqrt(T x);
template <>
__device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }
template <>
__device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }

// Fraction of the pixel [x - D/2, x + D/2] inside [a, b] (§2.2.2, Eq. 4).
template <typename T>
__device__ __forceinline__ T overlap(T x, T a, T b, T D, T invD) {
  T hi = fmin(b, x + T(0.5) * D);
  T lo = fmax(a, x - T(0.5) * D);
  T o = hi - lo;
  return o > T(0) ? o * invD : T(0);
}

// Depth-dose table lookup, linear, clamped at both ends; `tab` in LDS.
template <typename T>
__device__ __forceinline__ T dd_lookup(const T* tab, int n, T inv_step, T W) {
  T x = W * inv_step;
  if (!(x > T(0))) return tab[0];
  if (x >= T(n - 1)) return tab[n - 1];
  int i = (int)x;
  T f = x - T(i);
  T a = tab[i];
  return a + f * (tab[i + 1] - a);
}

// Trilinear density sample from the z-fastest copy rho_t [ny][nx][nz] at
// continuous voxel index (X, Y, Z), zero outside the CT.
template <typename T>
__device__ __forceinline__ T sample_rho(const T* __restrict__ rho_t, int nx, int ny, int nz, T X, T Y, T Z) {
  T fx0 = dfloor(X), fy0 = dfloor(Y), fz0 = dfloor(Z);
  int x0 = (int)fx0, y0 = (int)fy0, z0 = (int)fz0;
  T wx = X - fx0, wy = Y - fy0, wz = Z - fz0;
  if (x0 < -1 || x0 >= nx || y0 < -1 || y0 >= ny || z0 < -1 || z0 >= nz) return T(0);
  bool zin0 = z0 >= 0, zin1 = z0 + 1 < nz;
  T s = T(0);
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    int y = y0 + dy;
    if (y < 0 || y >= ny) continue;
    T wyv = dy ? wy : T(1) - wy;
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      int x = x0 + dx;
      if (x < 0 || x >= nx) continue;
      T wxv = dx ? wx : T(1) - wx;
      const T* col = rho_t + ((size_t)y * nx + x) * nz;
      T a = zin0 ? col[z0] : T(0);
      T b = zin1 ? col[z0 + 1] : T(0);
      s += wyv * wxv * (a + wz * (b - a));
    }
  }
  return s;
}

// Map a voxel (relative position t to the isocentre) into continuous beam-frame
// indices (kappa, iota, jota) for a control point with frame (sn, cs) (§2.2.7).
template <typename T>
struct FanIdx {
  T k, i, j;
};

template <typename T>
__device__ __forceinline__ FanIdx<T> voxel_to_fan(const Geo<T>& g, T sn, T cs, T tx, T ty, T tz) {
  T e = -sn * tx + cs * ty;             // d - SAD
  T q = T(1) / (T(1) + e * g.inv_sad);  // SAD / d
  T u = (cs * tx + sn * ty) * q;
  T v = tz * q;
  FanIdx<T> r;
  r.k = (e - g.e0) * g.inv_dstep;
  r.i = u * g.inv_lat + g.cu;
  r.j = v * g.inv_lat + g.cv;
  return r;
}

}  // namespace pdrt
