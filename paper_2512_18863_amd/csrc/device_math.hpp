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

// Depth-dose table lookup, linear, clamped at both ends; `tab` in LDS.  Branch
// free; at and below zero the interpolation weight is exactly 0 (tab[0]), at and
// beyond the last entry the 0/1 blend returns tab[n-1] exactly.
template <typename T>
__device__ __forceinline__ T dd_lookup(const T* tab, int n, T inv_step, T W) {
  const T x = W * inv_step;
  const T xc = fmin(fmax(x, T(0)), T(n - 1));  // NaN -> 0
  const int i = min((int)xc, n - 2);
  const T f = xc - T(i);
  const T a = tab[i];
  const T v = a + f * (tab[i + 1] - a);
  const T hi = T(x >= T(n - 1));  // 0/1 factors keep the table reads unconditional
  return (T(1) - hi) * v + hi * tab[n - 1];
}

// Trilinear density sample from the z-fastest copy rho_t [ny][nx][nz] at
// continuous voxel index (X, Y, Z), zero outside the CT, split in two halves: the
// fetch issues the eight corner loads from clamped (always valid) addresses, the
// combine masks and sums them in the order a masked loop would.  A ray march can
// fetch a few samples ahead, so several samples' loads are in flight together.
template <typename T>
struct RhoFetch {
  T lo[2][2], hi[2][2];
  T wx, wy, wz;
  T m_in, m_z0, m_z1, m_ok[2][2];  // 0/1 masks
};

template <typename T>
__device__ __forceinline__ RhoFetch<T> rho_fetch(const T* __restrict__ rho_t, int nx, int ny, int nz, T X, T Y, T Z) {
  RhoFetch<T> r;
  const T fx0 = dfloor(X), fy0 = dfloor(Y), fz0 = dfloor(Z);
  // (bitwise & keeps the flags branch free)
  const bool inside = (fx0 >= T(-1)) & (fx0 < T(nx)) & (fy0 >= T(-1)) & (fy0 < T(ny)) & (fz0 >= T(-1)) &
                      (fz0 < T(nz));
  const int x0 = inside ? (int)fx0 : 0, y0 = inside ? (int)fy0 : 0, z0 = inside ? (int)fz0 : 0;
  r.wx = X - fx0;
  r.wy = Y - fy0;
  r.wz = Z - fz0;
  r.m_in = T(inside);
  r.m_z0 = T(z0 >= 0);
  r.m_z1 = T(z0 + 1 < nz);
  const int za = max(z0, 0), zb = min(z0 + 1, nz - 1);
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const int y = y0 + dy, x = x0 + dx;
      r.m_ok[dy][dx] = T((y >= 0) & (y < ny) & (x >= 0) & (x < nx));
      const int cy = min(max(y, 0), ny - 1), cx = min(max(x, 0), nx - 1);
      const T* col = rho_t + (cy * nx + cx) * nz;  // (the volume holds fewer than 2^31 voxels)
      r.lo[dy][dx] = col[za];
      r.hi[dy][dx] = col[zb];
    }
  return r;
}

// Masks are 0/1 factors rather than selects (the clamped corners hold finite
// densities), so the compiler has no reason to make the loads conditional.
template <typename T>
__device__ __forceinline__ T rho_combine(const RhoFetch<T>& r) {
  T s = T(0);
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    const T wyv = dy ? r.wy : T(1) - r.wy;
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const T wxv = dx ? r.wx : T(1) - r.wx;
      const T a = r.m_z0 * r.lo[dy][dx];
      const T b = r.m_z1 * r.hi[dy][dx];
      s += r.m_ok[dy][dx] * (wyv * wxv * (a + r.wz * (b - a)));
    }
  }
  return r.m_in * s;
}

template <typename T>
__device__ __forceinline__ T sample_rho(const T* __restrict__ rho_t, int nx, int ny, int nz, T X, T Y, T Z) {
  return rho_combine(rho_fetch(rho_t, nx, ny, nz, X, Y, Z));
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
