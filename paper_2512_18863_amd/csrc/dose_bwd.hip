// dose_bwd.hip — reverse-mode kernels of the dose path and the projection layer.
//
// Given g = dL/dD the backward of one control-point batch runs
//   k_backproject_adj  Ghat_b = (trilinear back-projection)^T g   (adjoint of §2.2.7)
//   conv          H = K_k (*) Ghat_k (the taps are point symmetric, so the
//                 transposed convolution is the convolution itself; §2.2.6)
//   k_march<ADJ>  A = sum_k H_k (SAD/d_k)^2 DD(W_k), W recomputed    (§2.2.3-2.2.4)
//   k_param_grad  dL/dMU = calib <A, F>, dL/dF = calib MU A, then the chain rule
//                 through the fluence map (§2.2.2) to leaves and jaws.
// Depth and kernels are outside the gradient graph (§2.1), so nothing flows to
// the density.
#include "device_math.hpp"

namespace pdrt {

template <typename T>
__device__ __forceinline__ T overlap_da(T x, T a, T b, T D, T invD) {
  T hi = fmin(b, x + T(0.5) * D), lo = fmax(a, x - T(0.5) * D);
  return (hi - lo > T(0) && a > x - T(0.5) * D) ? -invD : T(0);
}
template <typename T>
__device__ __forceinline__ T overlap_db(T x, T a, T b, T D, T invD) {
  T hi = fmin(b, x + T(0.5) * D), lo = fmax(a, x - T(0.5) * D);
  return (hi - lo > T(0) && b < x + T(0.5) * D) ? invD : T(0);
}

// ------------------------------------------------------------------ adjoint of the back-projection

// Ghat_b = G_b^T g, where G_b is the trilinear back-projection of control point b
// (§2.2.7), computed in gather form: one wavefront per beam-frame column (k, i),
// lanes along v.  A voxel contributes to node (k, i, j) iff its continuous indices
// fall in [k-1, k+1) x [i-1, i+1) x [j-1, j+1); (kappa, iota) depend only on the
// voxel's (x, y) column, jota is increasing in z.  The wavefront bounds the
// candidate voxel columns by the rotated box around the trapezoid of beam-frame
// points with kappa, iota in range, evaluates each candidate with the forward's
// own index arithmetic, and for each lane walks the few z values whose jota lies
// in [j-1, j+1).  No atomics: every node is written once, summation order fixed.
// g_t is the dose gradient in z-fastest order [ny][nx][nz].
template <typename T, int NCH>
__global__ void __launch_bounds__(256) k_backproject_adj(Geo<T> g, const T* __restrict__ frame,
                                                         const T* __restrict__ g_t, T* __restrict__ Ghat) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + wave;
  const int b = blockIdx.y;
  if (col >= g.Nk * g.Nu) return;
  const int k = col / g.Nu, i = col - k * g.Nu;
  const T sn = frame[2 * b], cs = frame[2 * b + 1];
  // beam-frame box: e = d - SAD in [e_{k-1}, e_{k+1}], lateral l = u d / SAD
  const T e_lo = g.e0 + T(k - 1) * g.dstep, e_hi = g.e0 + T(k + 1) * g.dstep;
  const T u_lo = (T(i - 1) - g.cu) * g.lat, u_hi = (T(i + 1) - g.cu) * g.lat;
  const T s_lo = T(1) + e_lo * g.inv_sad, s_hi = T(1) + e_hi * g.inv_sad;
  const T l_lo = fmin(u_lo * s_lo, u_lo * s_hi), l_hi = fmax(u_hi * s_lo, u_hi * s_hi);
  T xmin = T(1e30), xmax = T(-1e30), ymin = T(1e30), ymax = T(-1e30);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    T e = (c & 1) ? e_hi : e_lo, l = (c & 2) ? l_hi : l_lo;
    T X = (-sn * e + cs * l - g.rel_ox) * g.inv_sx;
    T Y = (cs * e + sn * l - g.rel_oy) * g.inv_sy;
    xmin = fmin(xmin, X);
    xmax = fmax(xmax, X);
    ymin = fmin(ymin, Y);
    ymax = fmax(ymax, Y);
  }
  T* out = Ghat + ((size_t)b * g.Nk + k) * ((size_t)g.Nu * g.Nv) + (size_t)i * g.Nv;
  // candidate voxel columns: centres inside the box, widened by a rounding margin
  const T eps = T(1e-3);
  const int x0 = max(0, (int)dfloor(xmin - eps) + 1), x1 = min(g.nx - 1, (int)dfloor(xmax + eps));
  const int y0 = max(0, (int)dfloor(ymin - eps) + 1), y1 = min(g.ny - 1, (int)dfloor(ymax + eps));
  T acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = T(0);
  for (int y = y0; y <= y1; ++y) {
    const T ty = g.rel_oy + T(y) * g.sy;
    for (int x = x0; x <= x1; ++x) {
      const T tx = g.rel_ox + T(x) * g.sx;
      FanIdx<T> f = voxel_to_fan(g, sn, cs, tx, ty, T(0));
      const T fk = dfloor(f.k), fi = dfloor(f.i);
      const int k0 = (int)fk, i0 = (int)fi;
      if ((k0 != k && k0 != k - 1) || (i0 != i && i0 != i - 1)) continue;
      const T wk = f.k - fk, wi = f.i - fi;
      const T w2 = (k0 == k ? T(1) - wk : wk) * (i0 == i ? T(1) - wi : wi);
      const T q = T(1) / (T(1) + (-sn * tx + cs * ty) * g.inv_sad);  // SAD / d, as in voxel_to_fan
      const T dq = T(1) + (-sn * tx + cs * ty) * g.inv_sad;          // d / SAD
      const T* gcol = g_t + ((size_t)y * g.nx + x) * g.nz;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int j = 64 * c + lane;
        if (64 * c >= g.Nv) break;
        // z with jota in [j-1, j+1), widened by one voxel each side
        const T za = ((T(j - 1) - g.cv) * g.lat * dq - g.rel_oz) * g.inv_sz;
        const T zb = ((T(j + 1) - g.cv) * g.lat * dq - g.rel_oz) * g.inv_sz;
        const int z0 = max(0, (int)dfloor(za) - 1), z1 = min(g.nz - 1, (int)dfloor(zb) + 1);
        T part = T(0);
        for (int z = z0; z <= z1; ++z) {
          const T tz = g.rel_oz + T(z) * g.sz;
          const T jj = tz * q * g.inv_lat + g.cv;
          const T fj = dfloor(jj);
          const int j0 = (int)fj;
          const T wj = jj - fj;
          const T w = j0 == j ? T(1) - wj : (j0 == j - 1 ? wj : T(0));
          part += w * gcol[z];
        }
        acc[c] += w2 * part;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int j = 64 * c + lane;
    if (j < g.Nv) out[j] = acc[c];
  }
}

template <typename T>
hipError_t launch_backproject_adj(const Geo<T>& g, int nb, const T* frame, const T* g_t, T* Ghat, hipStream_t s) {
  dim3 grid((g.Nk * g.Nu + 3) / 4, nb);
  int nch = (g.Nv + 63) / 64;
  if (nch <= 1)
    hipLaunchKernelGGL((k_backproject_adj<T, 1>), grid, dim3(256), 0, s, g, frame, g_t, Ghat);
  else if (nch <= 2)
    hipLaunchKernelGGL((k_backproject_adj<T, 2>), grid, dim3(256), 0, s, g, frame, g_t, Ghat);
  else if (nch <= 4)
    hipLaunchKernelGGL((k_backproject_adj<T, 4>), grid, dim3(256), 0, s, g, frame, g_t, Ghat);
  else if (nch <= 8)
    hipLaunchKernelGGL((k_backproject_adj<T, 8>), grid, dim3(256), 0, s, g, frame, g_t, Ghat);
  else if (nch <= 16)
    hipLaunchKernelGGL((k_backproject_adj<T, 16>), grid, dim3(256), 0, s, g, frame, g_t, Ghat);
  else
    hipLaunchKernelGGL((k_backproject_adj<T, 64>), grid, dim3(256), 0, s, g, frame, g_t, Ghat);
  return hipGetLastError();
}

// ------------------------------------------------------------------ parameter gradients

template <typename T, int N>
__device__ void block_reduce(T (&v)[N], T* red) {
  int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < N; ++q) red[q * 256 + tid] = v[q];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
#pragma unroll
      for (int q = 0; q < N; ++q) red[q * 256 + tid] += red[q * 256 + tid + off];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = red[q * 256];
}

// One block per control point.  With F = fx fy [tau S + (1 - tau) O] and
// O = sum_l w_l f(u; l_l, r_l):
//   dL/dMU = calib sum A F,  gF = calib MU A,
//   dL/dx1 = sum gF dfx/dx1 fy [..]  (likewise x2, y1, y2),
//   dL/dl_l = sum gF fx fy (1 - tau) w_l df/dl_l  (likewise r_l),
// with the one-sided derivatives of the overlap (strict inequalities).
// Sums are fixed-order (tree reductions, per-edge loops): deterministic.
template <typename T>
__global__ void __launch_bounds__(256) k_param_grad(Geo<T> g, const T* __restrict__ leaves,
                                                    const T* __restrict__ jaws, const T* __restrict__ mu,
                                                    const T* __restrict__ A, T* __restrict__ gleaves,
                                                    T* __restrict__ gjaws, T* __restrict__ gmu) {
  __shared__ T red[5 * 256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int plane = g.Nu * g.Nv, L = g.L;
  const T D = g.lat, iD = g.inv_lat, tau = g.tau;
  const T* jw = jaws + 4 * b;
  const T* lv = leaves + (size_t)2 * L * b;
  const T* Ab = A + (size_t)b * plane;
  const T scale = g.calib * mu[b];
  T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
  for (int r = tid; r < plane; r += 256) {
    int i = r / g.Nv, j = r - i * g.Nv;
    T u = (T(i) - g.cu) * D, v = (T(j) - g.cv) * D;
    T fx = overlap(u, jw[0], jw[1], D, iD), fy = overlap(v, jw[2], jw[3], D, iD);
    T dx1 = overlap_da(u, jw[0], jw[1], D, iD), dx2 = overlap_db(u, jw[0], jw[1], D, iD);
    T dy1 = overlap_da(v, jw[2], jw[3], D, iD), dy2 = overlap_db(v, jw[2], jw[3], D, iD);
    if (fx == T(0) && fy == T(0)) continue;
    if (fx == T(0) && dx1 == T(0) && dx2 == T(0)) continue;
    if (fy == T(0) && dy1 == T(0) && dy2 == T(0)) continue;
    T S = T(0), O = T(0);
    for (int l = 0; l < L; ++l) {
      T w = overlap(v, g.leaf_edges[l], g.leaf_edges[l + 1], D, iD);
      if (w > T(0)) {
        S += w;
        O += w * overlap(u, lv[l], lv[L + l], D, iD);
      }
    }
    T br = tau * S + (T(1) - tau) * O;
    T a = Ab[r];
    T gF = scale * a;
    acc[0] += a * fx * fy * br;
    acc[1] += gF * dx1 * fy * br;
    acc[2] += gF * dx2 * fy * br;
    acc[3] += gF * fx * dy1 * br;
    acc[4] += gF * fx * dy2 * br;
  }
  block_reduce<T, 5>(acc, red);
  if (tid == 0) {
    gmu[b] = g.calib * acc[0];
    for (int q = 0; q < 4; ++q) gjaws[4 * b + q] = acc[1 + q];
  }
  for (int t = tid; t < 2 * L; t += 256) {
    int side = t / L, l = t - side * L;
    T lo = lv[l], hi = lv[L + l];
    T s = T(0);
    for (int j = 0; j < g.Nv; ++j) {
      T v = (T(j) - g.cv) * D;
      T w = overlap(v, g.leaf_edges[l], g.leaf_edges[l + 1], D, iD);
      if (!(w > T(0))) continue;
      T fy = overlap(v, jw[2], jw[3], D, iD);
      if (fy == T(0)) continue;
      for (int i = 0; i < g.Nu; ++i) {
        T u = (T(i) - g.cu) * D;
        T d = side ? overlap_db(u, lo, hi, D, iD) : overlap_da(u, lo, hi, D, iD);
        if (d == T(0)) continue;
        T fx = overlap(u, jw[0], jw[1], D, iD);
        s += scale * Ab[(size_t)i * g.Nv + j] * fx * fy * (T(1) - tau) * w * d;
      }
    }
    gleaves[(size_t)2 * L * b + t] = s;
  }
}

template <typename T>
hipError_t launch_param_grad(const Geo<T>& g, int nb, const T* leaves, const T* jaws, const T* mu, const T* A,
                             T* gleaves, T* gjaws, T* gmu, hipStream_t s) {
  hipLaunchKernelGGL(k_param_grad<T>, dim3(nb), dim3(256), 0, s, g, leaves, jaws, mu, A, gleaves, gjaws, gmu);
  return hipGetLastError();
}

// ------------------------------------------------------------------ projection (§2.2.1)

struct Limits {
  float leaf, jx, jy, w_min, mu_min;
};

__device__ __forceinline__ void project_pair(float a, float b, float lim, float w_min, float* oa, float* ob) {
  float c = 0.5f * (a + b), w = b - a;
  w = fmaxf(w, w_min);
  c = fminf(fmaxf(c, -lim), lim);
  *oa = c - 0.5f * w;
  *ob = c + 0.5f * w;
}

__global__ void k_project(int n_cp, int L, const float* __restrict__ lv, const float* __restrict__ jw,
                          const float* __restrict__ mu, Limits lim, float* lo, float* jo, float* mo) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int per = L + 3;  // leaf pairs, two jaw pairs, MU
  if (t >= n_cp * per) return;
  int b = t / per, q = t - b * per;
  if (q < L) {
    float a = lv[(size_t)2 * L * b + q], c = lv[(size_t)2 * L * b + L + q], oa, ob;
    project_pair(a, c, lim.leaf, lim.w_min, &oa, &ob);
    lo[(size_t)2 * L * b + q] = oa;
    lo[(size_t)2 * L * b + L + q] = ob;
  } else if (q < L + 2) {
    int p = q - L;
    float a = jw[4 * b + 2 * p], c = jw[4 * b + 2 * p + 1], oa, ob;
    project_pair(a, c, p ? lim.jy : lim.jx, lim.w_min, &oa, &ob);
    jo[4 * b + 2 * p] = oa;
    jo[4 * b + 2 * p + 1] = ob;
  } else {
    mo[b] = fmaxf(mu[b], lim.mu_min);
  }
}

// Jacobian of project_pair: a' = c' - w'/2, b' = c' + w'/2 with dc'/dc = [|c| < lim],
// dw'/dw = [w > w_min]; c = (a + b)/2, w = b - a.
__device__ __forceinline__ void project_pair_bwd(float a, float b, float lim, float w_min, float ga, float gb,
                                                 float* oa, float* ob) {
  float c = 0.5f * (a + b), w = b - a;
  float dc = (c > -lim && c < lim) ? 1.f : 0.f;
  float dw = (w > w_min) ? 1.f : 0.f;
  *oa = 0.5f * (dc + dw) * ga + 0.5f * (dc - dw) * gb;
  *ob = 0.5f * (dc - dw) * ga + 0.5f * (dc + dw) * gb;
}

__global__ void k_project_bwd(int n_cp, int L, const float* __restrict__ lv, const float* __restrict__ jw,
                              const float* __restrict__ mu, Limits lim, int ste, const float* gl, const float* gj,
                              const float* gm, float* ol, float* oj, float* om) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int per = L + 3;
  if (t >= n_cp * per) return;
  int b = t / per, q = t - b * per;
  if (q < L) {
    size_t ia = (size_t)2 * L * b + q, ib = ia + L;
    float ga = gl[ia], gb = gl[ib], oa = ga, ob = gb;
    if (!ste) project_pair_bwd(lv[ia], lv[ib], lim.leaf, lim.w_min, ga, gb, &oa, &ob);
    ol[ia] = oa;
    ol[ib] = ob;
  } else if (q < L + 2) {
    int p = q - L;
    int ia = 4 * b + 2 * p, ib = ia + 1;
    float ga = gj[ia], gb = gj[ib], oa = ga, ob = gb;
    if (!ste) project_pair_bwd(jw[ia], jw[ib], p ? lim.jy : lim.jx, lim.w_min, ga, gb, &oa, &ob);
    oj[ia] = oa;
    oj[ib] = ob;
  } else {
    om[b] = (ste || mu[b] > lim.mu_min) ? gm[b] : 0.f;
  }
}

hipError_t launch_project(int n_cp, int L, const float* lv, const float* jw, const float* mu, double leaf_lim,
                          double jx_lim, double jy_lim, double w_min, double mu_min, float* lo, float* jo, float* mo,
                          hipStream_t s) {
  Limits lim{(float)leaf_lim, (float)jx_lim, (float)jy_lim, (float)w_min, (float)mu_min};
  int n = n_cp * (L + 3);
  hipLaunchKernelGGL(k_project, dim3((n + 255) / 256), dim3(256), 0, s, n_cp, L, lv, jw, mu, lim, lo, jo, mo);
  return hipGetLastError();
}

hipError_t launch_project_bwd(int n_cp, int L, const float* lv, const float* jw, const float* mu, double leaf_lim,
                              double jx_lim, double jy_lim, double w_min, double mu_min, int ste, const float* gl,
                              const float* gj, const float* gm, float* ol, float* oj, float* om, hipStream_t s) {
  Limits lim{(float)leaf_lim, (float)jx_lim, (float)jy_lim, (float)w_min, (float)mu_min};
  int n = n_cp * (L + 3);
  hipLaunchKernelGGL(k_project_bwd, dim3((n + 255) / 256), dim3(256), 0, s, n_cp, L, lv, jw, mu, lim, ste, gl, gj,
                     gm, ol, oj, om);
  return hipGetLastError();
}

template hipError_t launch_backproject_adj<float>(const Geo<float>&, int, const float*, const float*, float*,
                                                  hipStream_t);
template hipError_t launch_backproject_adj<double>(const Geo<double>&, int, const double*, const double*, double*,
                                                   hipStream_t);
template hipError_t launch_param_grad<float>(const Geo<float>&, int, const float*, const float*, const float*,
                                             const float*, float*, float*, float*, hipStream_t);
template hipError_t launch_param_grad<double>(const Geo<double>&, int, const double*, const double*, const double*,
                                              const double*, double*, double*, double*, hipStream_t);

}  // namespace pdrt
