// fluence_corr.hip — fluence corrections of the fluence-generation layer
// (arXiv:2512.18863 §2.2.2 list): source penumbra, head scatter and the
// off-axis factor, applied to the aperture fluence maps [b][Nu][Nv] of a
// control-point batch, and their adjoint for the backward.
//
// Forward  Fc = O (F1 + a G_h F1),  F1 = G_v G_u F
// Adjoint  A^ = G_u G_v (X + a G_hu G_hv X),  X = O A
// with G_* separable unit-sum Gaussians (even taps, zero padding: each is its
// own transpose) and O the pointwise off-axis factor.  Every blur is one pass
// along one axis; the maps are small (180 x 89 x 89 at 128^3), so these are a
// few microseconds of memory traffic each.
#include "pdrt_internal.hpp"

namespace pdrt {

// out[b][i][j] = sum_m taps[m] in[b][i + m][j] (axis 0, along u) or
// in[b][i][j + m] (axis 1, along v), zero outside the map.
template <typename T>
__global__ void __launch_bounds__(256) k_blur(int nb, int Nu, int Nv, int axis, BlurTaps<T> t,
                                              const T* __restrict__ in, T* __restrict__ out) {
  const size_t plane = (size_t)Nu * Nv;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= plane * nb) return;
  const size_t b = q / plane;
  const int r = (int)(q - b * plane);
  const int i = r / Nv, j = r - i * Nv;
  const T* src = in + b * plane;
  T acc = T(0);
  if (axis == 0) {
    for (int m = -t.R; m <= t.R; ++m) {
      const int ii = i + m;
      if (ii >= 0 && ii < Nu) acc += t.g[m + t.R] * src[(size_t)ii * Nv + j];
    }
  } else {
    for (int m = -t.R; m <= t.R; ++m) {
      const int jj = j + m;
      if (jj >= 0 && jj < Nv) acc += t.g[m + t.R] * src[(size_t)i * Nv + jj];
    }
  }
  out[q] = acc;
}

// out = (x + a y) * (use_oar ? 1 + oar0 r + oar1 r^2 : 1), r the pixel's distance
// from the central axis at the isocentre plane.  out may alias x or y.
template <typename T>
__global__ void __launch_bounds__(256) k_fcorr_combine(int nb, int Nu, int Nv, T cu, T cv, T lat, T a, int use_oar,
                                                       T oar0, T oar1, const T* x, const T* y, T* out) {
  const size_t plane = (size_t)Nu * Nv;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= plane * nb) return;
  const int r = (int)(q % plane);
  const int i = r / Nv, j = r - i * Nv;
  T v = x[q] + a * y[q];
  if (use_oar) {
    const T u = (T(i) - cu) * lat, w = (T(j) - cv) * lat;
    const T rr = sqrt(u * u + w * w);
    v *= T(1) + oar0 * rr + oar1 * rr * rr;
  }
  out[q] = v;
}

template <typename T>
hipError_t launch_blur(const Geo<T>& g, int nb, int axis, const BlurTaps<T>& t, const T* in, T* out, hipStream_t s) {
  const size_t n = (size_t)g.Nu * g.Nv * nb;
  hipLaunchKernelGGL(k_blur<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nb, g.Nu, g.Nv, axis, t, in, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fcorr_combine(const Geo<T>& g, int nb, T a, int use_oar, const T* x, const T* y, T* out,
                                hipStream_t s) {
  const size_t n = (size_t)g.Nu * g.Nv * nb;
  hipLaunchKernelGGL(k_fcorr_combine<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nb, g.Nu, g.Nv, g.cu,
                     g.cv, g.lat, a, use_oar, g.oar0, g.oar1, x, y, out);
  return hipGetLastError();
}

#define PDRT_FC_INST(T)                                                                                         \
  template hipError_t launch_blur<T>(const Geo<T>&, int, int, const BlurTaps<T>&, const T*, T*, hipStream_t);   \
  template hipError_t launch_fcorr_combine<T>(const Geo<T>&, int, T, int, const T*, const T*, T*, hipStream_t);

PDRT_FC_INST(float)
PDRT_FC_INST(double)

}  // namespace pdrt
