// collimator.hip — collimator rotation of the fluence map (arXiv:2512.18863
// §2.2.2, last paragraph): the map rasterised in the collimator frame (leaves
// along u, stacked along v) is turned about the central axis by the collimator
// angle before the rays are traced.
//
// Beam-frame pixel (i, j) at (u, v) = ((i - cu) D, (j - cv) D) takes the
// collimator-frame map at (u', v') = (c u + s v, -s u + c v), (s, c) = (sin, cos)
// of the collimator angle, sampled bilinearly between pixel centres with zero
// outside the grid.  The adjoint is the transpose of that sampling, computed in
// gather form: each collimator-frame pixel sums the beam-frame pixels whose
// sample point lies within one pixel of it, with the forward's own weights, in a
// fixed order (no atomics, deterministic).  Maps are [b][Nu][Nv], v fastest.
#include "pdrt_internal.hpp"

namespace pdrt {

// Continuous collimator-frame pixel index of beam-frame pixel (i, j).
template <typename T>
__device__ __forceinline__ void coll_sample(const Geo<T>& g, T sn, T cs, int i, int j, T* ci, T* cj) {
  const T u = (T(i) - g.cu) * g.lat, v = (T(j) - g.cv) * g.lat;
  *ci = (cs * u + sn * v) * g.inv_lat + g.cu;
  *cj = (-sn * u + cs * v) * g.inv_lat + g.cv;
}

template <typename T>
__global__ void __launch_bounds__(256) k_rotate(Geo<T> g, int nb, const T* __restrict__ cframe,
                                                const T* __restrict__ Fc, T* __restrict__ Fb) {
  const size_t plane = (size_t)g.Nu * g.Nv;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= plane * nb) return;
  const int b = (int)(q / plane);
  const int r = (int)(q - (size_t)b * plane);
  const int i = r / g.Nv, j = r - i * g.Nv;
  T ci, cj;
  coll_sample(g, cframe[2 * b], cframe[2 * b + 1], i, j, &ci, &cj);
  if (!(fabs(ci) < T(1e8)) || !(fabs(cj) < T(1e8))) {
    Fb[q] = ci - ci + cj;  // non-finite angle: NaN propagates
    return;
  }
  const T fi0 = floor(ci), fj0 = floor(cj);
  const int i0 = (int)fi0, j0 = (int)fj0;
  const T fi = ci - fi0, fj = cj - fj0;
  const T* src = Fc + (size_t)b * plane;
  T acc = T(0);
#pragma unroll
  for (int di = 0; di < 2; ++di) {
    const int ii = i0 + di;
    if (ii < 0 || ii >= g.Nu) continue;
    const T wi = di ? fi : T(1) - fi;
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
      const int jj = j0 + dj;
      if (jj < 0 || jj >= g.Nv) continue;
      const T wj = dj ? fj : T(1) - fj;
      acc += (wi * wj) * src[(size_t)ii * g.Nv + jj];
    }
  }
  Fb[q] = acc;
}

// gFc[p] = sum_q w(q, p) A[q].  Beam pixel q reaches corner p iff p_i is floor(ci)
// or floor(ci) + 1 (likewise j), i.e. its sample lies in [p - 1, p + 1); those q lie
// within sqrt(2) pixels of p turned back into the beam frame, so the candidates are
// the pixels within 1.5 of that point along each axis.
template <typename T>
__global__ void __launch_bounds__(256) k_rotate_adj(Geo<T> g, int nb, const T* __restrict__ cframe,
                                                    const T* __restrict__ A, T* __restrict__ gFc) {
  const size_t plane = (size_t)g.Nu * g.Nv;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= plane * nb) return;
  const int b = (int)(q / plane);
  const int r = (int)(q - (size_t)b * plane);
  const int pi = r / g.Nv, pj = r - pi * g.Nv;
  const T sn = cframe[2 * b], cs = cframe[2 * b + 1];
  const T di = T(pi) - g.cu, dj = T(pj) - g.cv;
  const T xi = cs * di - sn * dj + g.cu, xj = sn * di + cs * dj + g.cv;
  if (!(fabs(xi) < T(1e8)) || !(fabs(xj) < T(1e8))) {
    gFc[q] = xi - xi + xj;
    return;
  }
  const int qi0 = max(0, (int)ceil(xi - T(1.5))), qi1 = min(g.Nu - 1, (int)floor(xi + T(1.5)));
  const int qj0 = max(0, (int)ceil(xj - T(1.5))), qj1 = min(g.Nv - 1, (int)floor(xj + T(1.5)));
  const T* Ab = A + (size_t)b * plane;
  T acc = T(0);
  for (int qi = qi0; qi <= qi1; ++qi)
    for (int qj = qj0; qj <= qj1; ++qj) {
      T ci, cj;
      coll_sample(g, sn, cs, qi, qj, &ci, &cj);
      const T fi0 = floor(ci), fj0 = floor(cj);
      const int i0 = (int)fi0, j0 = (int)fj0;
      const T fi = ci - fi0, fj = cj - fj0;
      const T wi = pi == i0 ? T(1) - fi : (pi == i0 + 1 ? fi : T(0));
      const T wj = pj == j0 ? T(1) - fj : (pj == j0 + 1 ? fj : T(0));
      if (wi != T(0) && wj != T(0)) acc += (wi * wj) * Ab[(size_t)qi * g.Nv + qj];
    }
  gFc[q] = acc;
}

// The aperture rectangle box[b] (collimator-frame pixel ranges [u0, u1) x [v0, v1)
// outside which the collimator-frame map and its derivatives vanish) becomes the
// beam-frame rectangle that holds every pixel whose bilinear sample reaches it:
// the rotated corners of the rectangle widened by one pixel, plus one pixel of
// margin for rounding, clipped to the grid.
template <typename T>
__global__ void k_collimator_box(Geo<T> g, int nb, const T* __restrict__ cframe, int* __restrict__ box) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int* bx = box + 4 * b;
  if (bx[1] <= bx[0] || bx[3] <= bx[2]) return;  // empty stays empty
  const T sn = cframe[2 * b], cs = cframe[2 * b + 1];
  if (!(fabs(sn) <= T(1)) || !(fabs(cs) <= T(1))) {
    bx[0] = 0, bx[1] = g.Nu, bx[2] = 0, bx[3] = g.Nv;
    return;
  }
  const T a[2] = {T(bx[0] - 1) - g.cu, T(bx[1]) - g.cu};
  const T c[2] = {T(bx[2] - 1) - g.cv, T(bx[3]) - g.cv};
  T xlo = T(1e30), xhi = T(-1e30), ylo = T(1e30), yhi = T(-1e30);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      const T x = cs * a[p] - sn * c[q] + g.cu, y = sn * a[p] + cs * c[q] + g.cv;
      xlo = fmin(xlo, x), xhi = fmax(xhi, x), ylo = fmin(ylo, y), yhi = fmax(yhi, y);
    }
  bx[0] = max(0, (int)floor(xlo) - 1);
  bx[1] = min(g.Nu, (int)ceil(xhi) + 2);
  bx[2] = max(0, (int)floor(ylo) - 1);
  bx[3] = min(g.Nv, (int)ceil(yhi) + 2);
  if (bx[1] < bx[0]) bx[1] = bx[0];
  if (bx[3] < bx[2]) bx[3] = bx[2];
}

template <typename T>
hipError_t launch_rotate(const Geo<T>& g, int nb, const T* cframe, const T* Fc, T* Fb, int adjoint, hipStream_t s) {
  const size_t n = (size_t)g.Nu * g.Nv * nb;
  if (adjoint)
    hipLaunchKernelGGL(k_rotate_adj<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, nb, cframe, Fc, Fb);
  else
    hipLaunchKernelGGL(k_rotate<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, nb, cframe, Fc, Fb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_collimator_box(const Geo<T>& g, int nb, const T* cframe, int* box, hipStream_t s) {
  hipLaunchKernelGGL(k_collimator_box<T>, dim3((nb + 63) / 64), dim3(64), 0, s, g, nb, cframe, box);
  return hipGetLastError();
}

#define PDRT_COLL_INST(T)                                                                                   \
  template hipError_t launch_rotate<T>(const Geo<T>&, int, const T*, const T*, T*, int, hipStream_t);       \
  template hipError_t launch_collimator_box<T>(const Geo<T>&, int, const T*, int*, hipStream_t);

PDRT_COLL_INST(float)
PDRT_COLL_INST(double)

}  // namespace pdrt
