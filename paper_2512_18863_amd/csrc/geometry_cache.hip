// geometry_cache.hip — the dose path with a plan-level geometry cache
// (arXiv:2512.18863 §2.2.3-2.2.4, Eqs. 6-7, used inside the optimisation loop of
// §2.5).
//
// While a plan is optimised only leaves, jaws and MU change; the density, the
// gantry angles and hence every ray's water-equivalent depth stay fixed.  The
// primary factorises as P_k(u, v) = F(u, v) G_k(u, v) with the aperture-free
// G_k = (SAD / d_k)^2 DD(W_k(u, v)), so G (and the central-axis depths z_k that
// set the kernel taps) can be computed once per plan by the ray march and kept in
// HBM for all control points.  Each forward then replaces the march by
//   k_apply_geometry   P[b][k] = F[b] G[b][k]
// and each backward replaces the adjoint march by
//   k_geometry_adjoint A[b] = sum_k H[b][k] G[b][k]   (the march's segments and order)
// With an FP32 cache both produce exactly the values of the march (the same
// products and the same sum order); a BF16 cache halves the bytes read and
// rounds G to 8 significant bits.
#include "device_math.hpp"

namespace pdrt {

namespace {

// Rays outside the control point's aperture rectangle (box, when given) are
// skipped as in the ray march: P is not read there, and A there is 0.
__device__ __forceinline__ bool outside_box(const int* box, int b, int r, int Nv) {
  if (!box) return false;
  const int i = r / Nv, j = r - i * Nv;
  const int* bx = box + 4 * b;
  return !(i >= bx[0] && i < bx[1] && j >= bx[2] && j < bx[3]);
}

template <typename E>
__global__ void __launch_bounds__(256) k_apply_geometry(int Nk, int Nv, int plane, const float* __restrict__ F,
                                                        const E* __restrict__ G, float* __restrict__ P,
                                                        const int* __restrict__ box) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= plane || outside_box(box, b, r, Nv)) return;
  const float Fv = F[(size_t)b * plane + r];
  const E* gb = G + (size_t)b * Nk * plane + r;
  float* pb = P + (size_t)b * Nk * plane + r;
  if (Fv == 0.f) {
    for (int k = 0; k < Nk; ++k) pb[(size_t)k * plane] = 0.f;
    return;
  }
#pragma unroll 4
  for (int k = 0; k < Nk; ++k) pb[(size_t)k * plane] = Fv * (float)gb[(size_t)k * plane];
}

template <typename E>
__global__ void __launch_bounds__(256) k_geometry_adjoint(int Nk, int nseg, int Nv, int plane,
                                                          const float* __restrict__ H,
                                                          const E* __restrict__ G, float* __restrict__ A,
                                                          const int* __restrict__ box) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= plane) return;
  if (outside_box(box, b, r, Nv)) {
    A[(size_t)b * plane + r] = 0.f;
    return;
  }
  const E* gb = G + (size_t)b * Nk * plane + r;
  const float* hb = H + (size_t)b * Nk * plane + r;
  // the march's order: each segment's fused multiply-adds in plane order, then the
  // segments' sums in segment order
  float a = 0.f;
  for (int w = 0; w < nseg; ++w) {
    float acc = 0.f;
#pragma unroll 4
    for (int k = (Nk * w) / nseg; k < (Nk * (w + 1)) / nseg; ++k)
      acc = fmaf(hb[(size_t)k * plane], (float)gb[(size_t)k * plane], acc);
    a += acc;
  }
  A[(size_t)b * plane + r] = a;
}

}  // namespace

template <typename E>
hipError_t launch_apply_geometry(const Geo<float>& g, int nb, const float* F, const E* G, float* P, hipStream_t s,
                                 const int* box) {
  const int plane = g.Nu * g.Nv;
  hipLaunchKernelGGL(k_apply_geometry<E>, dim3((plane + 255) / 256, nb), dim3(256), 0, s, g.Nk, g.Nv, plane, F, G, P,
                     box);
  return hipGetLastError();
}

template <typename E>
hipError_t launch_geometry_adjoint(const Geo<float>& g, int nb, const float* H, const E* G, float* A, hipStream_t s,
                                   const int* box) {
  const int plane = g.Nu * g.Nv;
  const int nseg = g.march_scan ? march_segments(g.Nk) : 1;
  hipLaunchKernelGGL(k_geometry_adjoint<E>, dim3((plane + 255) / 256, nb), dim3(256), 0, s, g.Nk, nseg, g.Nv, plane,
                     H, G, A, box);
  return hipGetLastError();
}

template hipError_t launch_apply_geometry<float>(const Geo<float>&, int, const float*, const float*, float*,
                                                 hipStream_t, const int*);
template hipError_t launch_apply_geometry<__bf16>(const Geo<float>&, int, const float*, const __bf16*, float*,
                                                  hipStream_t, const int*);
template hipError_t launch_geometry_adjoint<float>(const Geo<float>&, int, const float*, const float*, float*,
                                                   hipStream_t, const int*);
template hipError_t launch_geometry_adjoint<__bf16>(const Geo<float>&, int, const float*, const __bf16*, float*,
                                                    hipStream_t, const int*);

}  // namespace pdrt
