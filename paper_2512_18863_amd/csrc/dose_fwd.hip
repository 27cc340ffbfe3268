// dose_fwd.hip — forward kernels of the dose path (arXiv:2512.18863 §2.2.2-2.2.7).
//
// Per control-point batch the forward runs
//   k_raster      fluence map F [b][Nu][Nv]                  (§2.2.2, Eq. 4)
//   k_ca_depth    central-axis depth z [b][Nk]               (§2.2.4, Eq. 7)
//   k_march       primary P = F (SAD/d)^2 DD(W) [b][Nk][Nu][Nv] (§2.2.3-2.2.4, Eqs. 6-7)
//   conv          beam-frame dose Dfan = K_k (*) P_k         (§2.2.5-2.2.6, Eq. 8)
//   k_gather      dose += MU_b trilinear(Dfan_b)             (§2.2.7, Eq. 9)
// k_frame and k_transpose_rho prepare per-call constants.
#include "taps.hpp"

namespace pdrt {

// ------------------------------------------------------------------ setup

template <typename T>
__global__ void k_frame(const T* __restrict__ gantry, int n_cp, T* __restrict__ frame) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_cp) return;
  double sn, cs;
  sincospi((double)gantry[b] / 180.0, &sn, &cs);
  frame[2 * b] = (T)sn;
  frame[2 * b + 1] = (T)cs;
}

template <typename T>
hipError_t launch_frame(const Geo<T>& g, const T* gantry, int n_cp, T* frame, hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_frame<T>, dim3((n_cp + 255) / 256), dim3(256), 0, s, gantry, n_cp, frame);
  return hipGetLastError();
}

struct HuTable {
  int n;
  float hu[16], rho[16];
};

// HU -> relative density: piecewise-linear calibration curve, clamped (§2.2).
__global__ void k_hu_to_density(long n, const float* __restrict__ hu, float* __restrict__ rho, HuTable t) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float h = hu[q];
  float r;
  if (h <= t.hu[0]) {
    r = t.rho[0];
  } else if (h >= t.hu[t.n - 1]) {
    r = t.rho[t.n - 1];
  } else {
    int s = 0;
    while (h > t.hu[s + 1]) ++s;
    float f = (h - t.hu[s]) / (t.hu[s + 1] - t.hu[s]);
    r = t.rho[s] + f * (t.rho[s + 1] - t.rho[s]);
  }
  rho[q] = r;
}

hipError_t launch_hu_to_density(long n, const float* hu, float* rho, int n_pts, const float* hp, const float* rp,
                                hipStream_t s) {
  HuTable t;
  t.n = n_pts;
  for (int i = 0; i < n_pts; ++i) {
    t.hu[i] = hp[i];
    t.rho[i] = rp[i];
  }
  hipLaunchKernelGGL(k_hu_to_density, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, hu, rho, t);
  return hipGetLastError();
}

// rho [nz][ny][nx] -> rho_t [ny][nx][nz] (per y slice, a tiled 2-D transpose).
template <typename T>
__global__ void __launch_bounds__(256) k_transpose_rho(int nx, int ny, int nz, const T* __restrict__ rho,
                                                        T* __restrict__ rho_t) {
  __shared__ T tile[32][33];
  int x0 = blockIdx.x * 32, z0 = blockIdx.y * 32, y = blockIdx.z;
  int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int z = z0 + r, x = x0 + tx;
    tile[r][tx] = (z < nz && x < nx) ? rho[((size_t)z * ny + y) * nx + x] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int x = x0 + r, z = z0 + tx;
    if (x < nx && z < nz) rho_t[((size_t)y * nx + x) * nz + z] = tile[tx][r];
  }
}

template <typename T>
hipError_t launch_transpose_rho(const Geo<T>& g, const T* rho, T* rho_t, hipStream_t s) {
  dim3 grid((g.nx + 31) / 32, (g.nz + 31) / 32, g.ny);
  hipLaunchKernelGGL(k_transpose_rho<T>, grid, dim3(256), 0, s, g.nx, g.ny, g.nz, rho, rho_t);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fluence

// Fluence map of one pixel (§2.2.2):
//   F = f(u; x1, x2) f(v; y1, y2) [tau S + (1 - tau) O],
//   S = sum_l w_l (row coverage by the leaf bank), O = sum_l w_l f(u; l_l, r_l).
template <typename T>
__global__ void __launch_bounds__(256) k_raster(Geo<T> g, const T* __restrict__ leaves, const T* __restrict__ jaws,
                                                T* __restrict__ F) {
  int b = blockIdx.y;
  int plane = g.Nu * g.Nv;
  int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= plane) return;
  int i = r / g.Nv, j = r - i * g.Nv;
  T D = g.lat, iD = g.inv_lat;
  T u = (T(i) - g.cu) * D, v = (T(j) - g.cv) * D;
  const T* jw = jaws + 4 * b;
  const T* lv = leaves + (size_t)2 * g.L * b;
  T fx = overlap(u, jw[0], jw[1], D, iD);
  T fy = overlap(v, jw[2], jw[3], D, iD);
  T S = T(0), O = T(0);
  if (fx * fy != T(0)) {
    for (int l = 0; l < g.L; ++l) {
      T w = overlap(v, g.leaf_edges[l], g.leaf_edges[l + 1], D, iD);
      if (w > T(0)) {
        S += w;
        O += w * overlap(u, lv[l], lv[g.L + l], D, iD);
      }
    }
  }
  F[(size_t)b * plane + r] = fx * fy * (g.tau * S + (T(1) - g.tau) * O);
}

template <typename T>
hipError_t launch_raster(const Geo<T>& g, int nb, const T* leaves, const T* jaws, T* F, hipStream_t s) {
  dim3 grid((g.Nu * g.Nv + 255) / 256, nb);
  hipLaunchKernelGGL(k_raster<T>, grid, dim3(256), 0, s, g, leaves, jaws, F);
  return hipGetLastError();
}

// Rectangle of fluence pixels [u0, u1) x [v0, v1) of each control point outside
// which F and all its derivatives are exactly zero: a pixel carries fluence only
// if it overlaps the jaw opening (the factor f(u; x1, x2) f(v; y1, y2) of Eq. 4),
// widened by one pixel for rounding and by (du, dv) pixels for the reach of the
// fluence corrections.  A non-finite jaw gives the whole plane.
template <typename T>
__device__ __forceinline__ void pixel_range(T a, T b, T c, int N, int d, T inv_lat, int* lo, int* hi) {
  const T fa = a * inv_lat + c - T(0.5), fb = b * inv_lat + c + T(0.5);
  if (!(fa == fa) || !(fb == fb) || !(fabs(fa) < T(1e8)) || !(fabs(fb) < T(1e8))) {
    *lo = 0;
    *hi = N;
    return;
  }
  int l = (int)floor(fa) - 1 - d, u = (int)ceil(fb) + 1 + d;
  l = max(l, 0);
  u = min(u, N);
  *lo = l;
  *hi = u > l ? u : l;
}

template <typename T>
__global__ void k_aperture_box(Geo<T> g, int nb, const T* __restrict__ jaws, int du, int dv, int* __restrict__ box) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const T* jw = jaws + 4 * b;
  int u0, u1, v0, v1;
  pixel_range(jw[0], jw[1], g.cu, g.Nu, du, g.inv_lat, &u0, &u1);
  pixel_range(jw[2], jw[3], g.cv, g.Nv, dv, g.inv_lat, &v0, &v1);
  box[4 * b] = u0;
  box[4 * b + 1] = u1;
  box[4 * b + 2] = v0;
  box[4 * b + 3] = v1;
}

template <typename T>
hipError_t launch_aperture_box(const Geo<T>& g, int nb, const T* jaws, int du, int dv, int* box, hipStream_t s) {
  hipLaunchKernelGGL(k_aperture_box<T>, dim3((nb + 63) / 64), dim3(64), 0, s, g, nb, jaws, du, dv, box);
  return hipGetLastError();
}

// ------------------------------------------------------------------ depth

// Central-axis depth (§2.2.4, Eq. 7): one wavefront per control point samples
// 64 consecutive planes at a time and turns them into the running integral with
// an inclusive wavefront prefix sum plus the carry of the previous chunk.
template <typename T>
__global__ void __launch_bounds__(64) k_ca_depth(Geo<T> g, const T* __restrict__ frame, const T* __restrict__ rho_t,
                                                 T* __restrict__ z) {
  int b = blockIdx.x;
  int lane = threadIdx.x;
  T sn = frame[2 * b], cs = frame[2 * b + 1];
  T carry = T(0);
  for (int k0 = 0; k0 < g.Nk; k0 += 64) {
    int k = k0 + lane;
    T val = T(0);
    if (k < g.Nk) {
      T e = g.e0 + T(k) * g.dstep;
      T X = g.iso_ix + (-e * sn) * g.inv_sx;
      T Y = g.iso_iy + (e * cs) * g.inv_sy;
      val = sample_rho(rho_t, g.nx, g.ny, g.nz, X, Y, g.iso_iz) * g.dstep;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      T o = __shfl_up(val, off, 64);
      if (lane >= off) val += o;
    }
    if (k < g.Nk) z[(size_t)b * g.Nk + k] = carry + val;
    carry += __shfl(val, 63, 64);
  }
}

template <typename T>
hipError_t launch_ca_depth(const Geo<T>& g, int nb, const T* frame, const T* rho_t, T* z, hipStream_t s) {
  hipLaunchKernelGGL(k_ca_depth<T>, dim3(nb), dim3(64), 0, s, g, frame, rho_t, z);
  return hipGetLastError();
}

// ------------------------------------------------------------------ ray march

// Ray (u_i, v_j) meets plane k at
//   q - iso = (d_k - SAD) b + (d_k / SAD)(u e_u + v e_v);
// the density is sampled trilinearly there, and the water-equivalent depth of
// Eq. 7 is the inclusive sum W_k = sum_{k' <= k} rho(q_k') ds, ds = Dd sqrt(1 +
// (u^2 + v^2)/SAD^2); the primary is P_k = F (SAD / d_k)^2 DD(W_k).
// MARCH_ADJOINT instead accumulates A = sum_k H_k (SAD / d_k)^2 DD(W_k) (the
// adjoint of the primary w.r.t. F); MARCH_GEOMETRY stores the aperture-independent
// factor G_k = (SAD / d_k)^2 DD(W_k) itself (rounded to E), so that P = F G later.
enum { MARCH_PRIMARY = 0, MARCH_ADJOINT = 1, MARCH_GEOMETRY = 2 };

// ---- serial form (the default)
//
// One thread per divergent ray (i, j) walks its Nk planes in order with a
// compensated running sum; eight planes' density loads are in flight at a time.
// Lanes run along v, i.e. along patient z, so the z-fastest density copy is read
// almost contiguously.  With a box (the aperture rectangle of each control point,
// given when the convolution honours it) rays outside it are skipped: the
// convolution never reads P there, and the adjoint's A there is written as 0
// (the parameter gradients only read it inside).
// One ray (i, j) of control point b.
template <typename T, int MODE, typename E>
__device__ __forceinline__ void march_ray(const Geo<T>& g, int b, int i, int j, const T* __restrict__ frame,
                                          const T* __restrict__ rho_t, const T* __restrict__ F,
                                          const T* __restrict__ zca, const T* tab, E* __restrict__ vol,
                                          T* __restrict__ A) {
  const int plane = g.Nu * g.Nv;
  const int r = i * g.Nv + j;
  E* vb = vol + (size_t)b * g.Nk * plane + r;
  T Fv = T(1);
  if (MODE == MARCH_PRIMARY) {
    Fv = F[(size_t)b * plane + r];
    if (Fv == T(0)) {
      for (int k = 0; k < g.Nk; ++k) vb[(size_t)k * plane] = E(0);
      return;
    }
  }
  T sn = frame[2 * b], cs = frame[2 * b + 1];
  T u = (T(i) - g.cu) * g.lat, v = (T(j) - g.cv) * g.lat;
  T ucs = u * cs, usn = u * sn;
  T ds = g.dstep * dsqrt(T(1) + (u * u + v * v) * (g.inv_sad * g.inv_sad));
  const T* zb = zca + (size_t)b * g.Nk;
  T W = T(0), c = T(0), acc = T(0);
  // one step of the march: the water-equivalent depth Wk of plane k, then the
  // primary (or its adjoint, or the factor itself) at that plane
  auto step = [&](int k, T Wk) {
    const T e = g.e0 + T(k) * g.dstep;
    const T gk = T(1) + e * g.inv_sad;
    const T geo = dd_lookup(tab, g.n_dd, g.inv_dd_step, Wk) / (gk * gk);
    if (MODE == MARCH_ADJOINT)
      acc = fma(T(vb[(size_t)k * plane]), geo, acc);
    else if (MODE == MARCH_PRIMARY)
      vb[(size_t)k * plane] = Fv * geo;
    else
      vb[(size_t)k * plane] = E(geo);
  };
  if (g.wepl_mode == PDRT_WEPL_PER_RAY) {
#pragma unroll 8
    for (int k = 0; k < g.Nk; ++k) {
      const T e = g.e0 + T(k) * g.dstep;
      const T gk = T(1) + e * g.inv_sad;
      const T X = g.iso_ix + (-e * sn + gk * ucs) * g.inv_sx;
      const T Y = g.iso_iy + (e * cs + gk * usn) * g.inv_sy;
      const T Z = g.iso_iz + (gk * v) * g.inv_sz;
      const T rho = sample_rho(rho_t, g.nx, g.ny, g.nz, X, Y, Z);
      const T y = rho * ds - c;  // Kahan-compensated running sum
      const T t = W + y;
      c = (t - W) - y;
      W = t;
      step(k, W);
    }
  } else {
    for (int k = 0; k < g.Nk; ++k) step(k, zb[k]);
  }
  if (MODE == MARCH_ADJOINT) A[(size_t)b * plane + r] = acc;
}

// Without a box, one thread per ray of the plane; with a box, the block row
// blockIdx.y = b walks only the rays of control point b's rectangle (grid-stride),
// so no lanes idle on rays outside it.  (In adjoint mode A outside the box is
// cleared beforehand.)
template <typename T, int MODE, typename E>
__global__ void __launch_bounds__(256) k_march_serial(Geo<T> g, const T* __restrict__ frame, const T* __restrict__ rho_t,
                                               const T* __restrict__ F, const T* __restrict__ zca,
                                               const T* __restrict__ dd, E* __restrict__ vol, T* __restrict__ A,
                                               const int* __restrict__ box) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  for (int q = threadIdx.x; q < g.n_dd; q += 256) tab[q] = dd[q];
  __syncthreads();
  const int b = blockIdx.y;
  if (box) {
    const int* bx = box + 4 * b;
    const int bw = bx[3] - bx[2], area = bx[1] > bx[0] && bw > 0 ? (bx[1] - bx[0]) * bw : 0;
    for (int rr = blockIdx.x * 256 + threadIdx.x; rr < area; rr += gridDim.x * 256) {
      const int li = rr / bw;
      march_ray<T, MODE, E>(g, b, bx[0] + li, bx[2] + rr - li * bw, frame, rho_t, F, zca, tab, vol, A);
    }
  } else {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < g.Nu * g.Nv) march_ray<T, MODE, E>(g, b, r / g.Nv, r % g.Nv, frame, rho_t, F, zca, tab, vol, A);
  }
}

// ---- segmented scan (spec->march_scan)
//
// The inclusive sum as a segmented scan across the wavefronts of a workgroup.
// The workgroup takes 64 rays (lanes along v, so that neighbouring lanes read
// neighbouring z of the z-fastest density copy) and its NW wavefronts take
// consecutive segments of the Nk planes: each wavefront samples its segment
// (samples kept in registers, MARCH_SEG planes per pass) and forms the segment's
// compensated sum; the segment sums go through LDS and each wavefront adds those
// of the segments before its own in plane order (its carry); it then rescans its
// segment from the carry, giving W_k for its planes, and applies the depth dose.
// In adjoint mode the wavefronts' partial sums of H_k (SAD/d_k)^2 DD(W_k) are
// added in LDS in segment order.  Every sum runs in a fixed order.
//
// With a box (the aperture rectangle of each control point, given when the
// convolution honours it) only the rays inside it are marched: the convolution
// never reads P outside it, and the adjoint's A there is written as 0 beforehand
// (the parameter gradients only read it inside).
constexpr int MARCH_SEG = kMarchSeg;           // planes per wavefront and pass
constexpr int MARCH_MAXW = kMarchMaxSegments;  // wavefronts per workgroup

template <typename T>
__device__ __forceinline__ void kahan_add(T& S, T& c, T x) {
  const T y = x - c;
  const T t = S + y;
  c = (t - S) - y;
  S = t;
}

template <typename T, int MODE, typename E>
__global__ void __launch_bounds__(64 * MARCH_MAXW) k_march_scan(Geo<T> g, const T* __restrict__ frame,
                                                           const T* __restrict__ rho_t, const T* __restrict__ F,
                                                           const T* __restrict__ zca, const T* __restrict__ dd,
                                                           E* __restrict__ vol, T* __restrict__ A,
                                                           const int* __restrict__ box) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* seg = reinterpret_cast<T*>(smem_raw);  // [2][MARCH_MAXW][64]: segment sums and compensations
  T* tab = seg + 2 * MARCH_MAXW * 64;       // depth-dose table [n_dd]
  const int nw = blockDim.x >> 6;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int q = tid; q < g.n_dd; q += blockDim.x) tab[q] = dd[q];
  __syncthreads();
  const int b = blockIdx.y;
  const int plane = g.Nu * g.Nv;
  int u0 = 0, nu = g.Nu, v0 = 0, nv = g.Nv;
  if (box) {
    const int* bx = box + 4 * b;
    u0 = bx[0], v0 = bx[2];
    nu = max(0, bx[1] - bx[0]), nv = max(0, bx[3] - bx[2]);
  }
  const int area = nu * nv;
  const int kb = (g.Nk * w) / nw, ke = (g.Nk * (w + 1)) / nw;  // this wavefront's planes
  const bool per_ray = g.wepl_mode == PDRT_WEPL_PER_RAY;
  const bool keep = ke - kb <= MARCH_SEG;  // one pass holds the whole segment
  const T sn = frame[2 * b], cs = frame[2 * b + 1];
  const T* zb = zca + (size_t)b * g.Nk;
  for (int grp = blockIdx.x; grp * 64 < area; grp += gridDim.x) {
    const int rr = grp * 64 + lane;
    const bool valid = rr < area;
    const int li = valid ? rr / nv : 0;
    const int i = u0 + li, j = v0 + (valid ? rr - li * nv : 0);
    const int r = i * g.Nv + j;
    const T u = (T(i) - g.cu) * g.lat, v = (T(j) - g.cv) * g.lat;
    const T ucs = u * cs, usn = u * sn;
    const T ds = g.dstep * dsqrt(T(1) + (u * u + v * v) * (g.inv_sad * g.inv_sad));
    // samples rho ds of planes k0 .. k0 + MARCH_SEG - 1 (zero past the segment),
    // four planes' corner loads issued together before they are combined
    T y[MARCH_SEG];
    auto sample_pass = [&](int k0) {
#pragma unroll
      for (int s0 = 0; s0 < MARCH_SEG; s0 += 4) {
        RhoFetch<T> fr[4];
#pragma unroll
        for (int s1 = 0; s1 < 4; ++s1) {
          const int k = min(k0 + s0 + s1, g.Nk - 1);
          const T e = g.e0 + T(k) * g.dstep;
          const T gk = T(1) + e * g.inv_sad;
          const T X = g.iso_ix + (-e * sn + gk * ucs) * g.inv_sx;
          const T Y = g.iso_iy + (e * cs + gk * usn) * g.inv_sy;
          const T Z = g.iso_iz + (gk * v) * g.inv_sz;
          fr[s1] = rho_fetch(rho_t, g.nx, g.ny, g.nz, X, Y, Z);
        }
#pragma unroll
        for (int s1 = 0; s1 < 4; ++s1)
          y[s0 + s1] = k0 + s0 + s1 < ke ? rho_combine(fr[s1]) * ds : T(0);
      }
    };
    T S = T(0), cS = T(0);
    if (per_ray) {
      for (int k0 = kb; k0 < ke; k0 += MARCH_SEG) {
        sample_pass(k0);
#pragma unroll
        for (int s2 = 0; s2 < MARCH_SEG; ++s2)
          if (k0 + s2 < ke) kahan_add(S, cS, y[s2]);
      }
      seg[w * 64 + lane] = S;
      seg[(MARCH_MAXW + w) * 64 + lane] = cS;
    }
    __syncthreads();
    // carry: the sums of the segments before this one, in plane order
    T W = T(0), cW = T(0);
    if (per_ray)
      for (int w2 = 0; w2 < w; ++w2) kahan_add(W, cW, seg[w2 * 64 + lane] - seg[(MARCH_MAXW + w2) * 64 + lane]);
    T Fv = T(1);
    if (MODE == MARCH_PRIMARY && valid) Fv = F[(size_t)b * plane + r];
    E* vb = vol + (size_t)b * g.Nk * plane + r;
    T acc = T(0);
    for (int k0 = kb; k0 < ke; k0 += MARCH_SEG) {
      if (per_ray && !keep) sample_pass(k0);
#pragma unroll
      for (int s2 = 0; s2 < MARCH_SEG; ++s2) {
        const int k = k0 + s2;
        if (k < ke) {
          T Wk;
          if (per_ray) {
            kahan_add(W, cW, y[s2]);
            Wk = W;
          } else {
            Wk = zb[k];
          }
          const T e = g.e0 + T(k) * g.dstep;
          const T gk = T(1) + e * g.inv_sad;
          const T geo = dd_lookup(tab, g.n_dd, g.inv_dd_step, Wk) / (gk * gk);
          if (valid) {
            if (MODE == MARCH_ADJOINT)
              acc = fma(T(vb[(size_t)k * plane]), geo, acc);
            else if (MODE == MARCH_PRIMARY)
              vb[(size_t)k * plane] = Fv * geo;
            else
              vb[(size_t)k * plane] = E(geo);
          }
        }
      }
    }
    if (MODE == MARCH_ADJOINT) {
      __syncthreads();
      seg[w * 64 + lane] = acc;
      __syncthreads();
      if (w == 0 && valid) {
        T a = T(0);
        for (int w2 = 0; w2 < nw; ++w2) a += seg[w2 * 64 + lane];
        A[(size_t)b * plane + r] = a;
      }
    }
    __syncthreads();  // the segment sums are reused by the next group
  }
}

template <typename T>
__global__ void k_fill_zero(size_t n, T* __restrict__ p) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
    p[q] = T(0);
}

// Workgroups per control point: enough for the 64-ray groups of the largest jaw
// rectangle the field limit allows (the plane minus the kernel halo, plus the
// rectangle's margins); the groups are walked grid-stride, so a larger rectangle
// (fluence corrections, collimator rotation, jaws beyond the field limit) is
// still covered.  Without a box, the groups of the whole plane.
template <typename T>
int march_groups(const Geo<T>& g, const int* box) {
  if (!box) return (g.Nu * g.Nv + 63) / 64;
  const int bu = min(g.Nu, g.Nu - 2 * g.h + 6), bv = min(g.Nv, g.Nv - 2 * g.h + 6);
  return max(1, (bu * bv + 63) / 64);
}

// Blocks per control point for the serial form with a box: enough for the
// largest jaw rectangle the field limit allows (the walk is grid-stride, so a
// larger box is still covered).
template <typename T>
int march_box_blocks(const Geo<T>& g) {
  const int bu = min(g.Nu, g.Nu - 2 * g.h + 6), bv = min(g.Nv, g.Nv - 2 * g.h + 6);
  return max(1, (bu * bv + 255) / 256);
}

// The scan's wavefronts per workgroup: segments of at most MARCH_SEG planes where
// eight wavefronts suffice (Nk <= 256), else eight segments of several passes.
template <typename T, int MODE, typename E>
hipError_t launch_march_mode(const Geo<T>& g, int nb, const T* frame, const T* rho_t, const T* F, const T* z,
                             const T* dd, E* vol, T* A, hipStream_t s, const int* box) {
  if (!g.march_scan) {
    dim3 grid(box ? march_box_blocks(g) : (g.Nu * g.Nv + 255) / 256, nb);
    hipLaunchKernelGGL((k_march_serial<T, MODE, E>), grid, dim3(256), g.n_dd * sizeof(T), s, g, frame, rho_t, F, z,
                       dd, vol, A, box);
    return hipGetLastError();
  }
  const int nw = march_segments(g.Nk);
  const size_t lds = sizeof(T) * (2 * MARCH_MAXW * 64 + (size_t)g.n_dd);
  if (lds > 64 * 1024) return hipErrorInvalidConfiguration;
  dim3 grid(march_groups(g, box), nb);
  hipLaunchKernelGGL((k_march_scan<T, MODE, E>), grid, dim3(64 * nw), lds, s, g, frame, rho_t, F, z, dd, vol, A,
                     box);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_march(const Geo<T>& g, int nb, const T* frame, const T* rho_t, const T* F, const T* z, const T* dd,
                        T* P, hipStream_t s, const int* box) {
  return launch_march_mode<T, MARCH_PRIMARY, T>(g, nb, frame, rho_t, F, z, dd, P, (T*)nullptr, s, box);
}

template <typename E>
hipError_t launch_march_geometry(const Geo<float>& g, int nb, const float* frame, const float* rho_t, const float* z,
                                 const float* dd, E* G, hipStream_t s) {
  return launch_march_mode<float, MARCH_GEOMETRY, E>(g, nb, frame, rho_t, (const float*)nullptr, z, dd, G,
                                                     (float*)nullptr, s, (const int*)nullptr);
}
template hipError_t launch_march_geometry<float>(const Geo<float>&, int, const float*, const float*, const float*,
                                                 const float*, float*, hipStream_t);
template hipError_t launch_march_geometry<__bf16>(const Geo<float>&, int, const float*, const float*, const float*,
                                                  const float*, __bf16*, hipStream_t);

template <typename T>
hipError_t launch_march_adj(const Geo<T>& g, int nb, const T* frame, const T* rho_t, const T* z, const T* dd,
                            const T* H, T* A, hipStream_t s, const int* box) {
  if (box) {
    const size_t n = (size_t)nb * g.Nu * g.Nv;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048)), dim3(256), 0,
                       s, n, A);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  }
  return launch_march_mode<T, MARCH_ADJOINT, T>(g, nb, frame, rho_t, (const T*)nullptr, z, dd, const_cast<T*>(H), A,
                                                s, box);
}

// ------------------------------------------------------------------ kernel taps

template <typename T>
__device__ void build_taps(const Geo<T>& g, int k, T zk, T* K, int tid, int nthreads) {
  TapParams<T> tp = tap_params(g, k, zk);
  int n = g.n_taps, h = g.h;
  for (int idx = tid; idx < n * n; idx += nthreads) K[idx] = tap_value(tp, idx / n - h, idx % n - h);
}

// ------------------------------------------------------------------ direct conv

// Zero-padded per-plane convolution Dfan_k = K_k (*) P_k (§2.2.6, Eq. 8) on the
// vector ALUs.  A block owns a 48 (u) x 32 (v) output tile of one plane; the
// input tile with its halo and the plane's taps are staged in LDS.  Each thread
// owns 6 outputs along u and slides a 6-deep register window down the tap rows,
// so each tap costs 6 FMAs per LDS load.  Used for the FP64 path and for small
// kernels.
constexpr int DC_COLS = 32, DC_RG = 8, DC_R = 6, DC_ROWS = DC_RG * DC_R;

template <typename T>
__global__ void __launch_bounds__(256) k_conv_direct(Geo<T> g, const T* __restrict__ zca, const T* __restrict__ in,
                                                     T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = g.n_taps, h = g.h;
  const int pitch = DC_COLS + 2 * h;
  const int rows = DC_ROWS + 2 * h + DC_R;  // DC_R spare rows for the window prefetch
  T* tile = reinterpret_cast<T*>(smem_raw);
  T* K = tile + rows * pitch;
  const int k = blockIdx.y, b = blockIdx.z;
  const int tiles_v = (g.Nv + DC_COLS - 1) / DC_COLS;
  const int i0 = (blockIdx.x / tiles_v) * DC_ROWS, j0 = (blockIdx.x % tiles_v) * DC_COLS;
  const int plane = g.Nu * g.Nv;
  const T* src = in + ((size_t)b * g.Nk + k) * plane;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < rows * pitch; idx += 256) {
    int rr = idx / pitch, cc = idx - rr * pitch;
    int i = i0 - h + rr, j = j0 - h + cc;
    T val = T(0);
    if (rr < DC_ROWS + 2 * h && i >= 0 && i < g.Nu && j >= 0 && j < g.Nv) val = src[(size_t)i * g.Nv + j];
    tile[idx] = val;
  }
  build_taps(g, k, zca[(size_t)b * g.Nk + k], K, tid, 256);
  __syncthreads();
  const int tx = tid % DC_COLS, ty = tid / DC_COLS;
  const int rbase = ty * DC_R;
  T acc[DC_R];
#pragma unroll
  for (int r = 0; r < DC_R; ++r) acc[r] = T(0);
  for (int q = 0; q < n; ++q) {
    const T* col = tile + rbase * pitch + tx + q;
    T w[DC_R];
#pragma unroll
    for (int r = 0; r < DC_R; ++r) w[r] = col[r * pitch];
    for (int p0 = 0; p0 < n; p0 += DC_R) {
#pragma unroll
      for (int s = 0; s < DC_R; ++s) {
        int p = p0 + s;
        if (p < n) {
          T t = K[p * n + q];
#pragma unroll
          for (int r = 0; r < DC_R; ++r) acc[r] += t * w[(r + s) % DC_R];
          w[s] = col[(p + DC_R) * pitch];
        }
      }
    }
  }
  T* dst = out + ((size_t)b * g.Nk + k) * plane;
  int j = j0 + tx;
#pragma unroll
  for (int r = 0; r < DC_R; ++r) {
    int i = i0 + rbase + r;
    if (i < g.Nu && j < g.Nv) dst[(size_t)i * g.Nv + j] = acc[r];
  }
}

template <typename T>
size_t conv_direct_lds(const Geo<T>& g) {
  int pitch = DC_COLS + 2 * g.h, rows = DC_ROWS + 2 * g.h + DC_R;
  return sizeof(T) * ((size_t)rows * pitch + (size_t)g.n_taps * g.n_taps);
}

template <typename T>
hipError_t launch_conv_direct(const Geo<T>& g, int nb, const T* z, const T* in, T* out, hipStream_t s) {
  size_t lds = conv_direct_lds(g);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  {
    hipError_t e = ensure_lds_limit((const void*)k_conv_direct<T>, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  int tiles = ((g.Nu + DC_ROWS - 1) / DC_ROWS) * ((g.Nv + DC_COLS - 1) / DC_COLS);
  dim3 grid(tiles, g.Nk, nb);
  hipLaunchKernelGGL(k_conv_direct<T>, grid, dim3(256), lds, s, g, z, in, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ gather

// Back-projection and MU-weighted sum (§2.2.7, Eq. 9).  One thread per voxel,
// lanes along z so the 2 x 2 beam-frame columns a wavefront reads are contiguous
// in v.  The sum over control points uses Neumaier compensation; across batches
// the running sum lives in `dose` and its compensation in `comp`.
//
// Workgroups are numbered so that each of the eight XCDs (which receive
// workgroups round robin) walks a contiguous range of y slabs: neighbouring voxel
// columns read the same beam-frame columns, and they then share one L2.
// The part of one control point's trilinear lookup that depends only on the
// voxel column (x, y): the beam-frame plane k and row i of the column (the same
// for every z), the four (k, i) corner weights with their in-grid masks and the
// corners' element offsets within the control point's beam-frame volume, and
// SAD / d, which scales z into the lateral coordinate j.
template <typename T>
struct GatherCol {
  T q;
  T w[4];     // corner (dk, di) = (c >> 1, c & 1): in-grid mask x (1 - wk or wk) x (1 - wi or wi)
  int off[4]; // element offset of the corner's row (clamped into the grid)
};

constexpr int GATHER_CHUNK = 64;  // control points whose column terms sit in LDS at once

// A wavefront-uniform value read from LDS, moved to scalar registers (so that
// addresses built from it use the scalar base of a global load).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// dose(x, y, z) += sum_b MU_b trilinear(Dfan_b at the voxel's beam-frame position).
// A block covers 64 consecutive z of a 4 x 4 patch of voxel columns (one
// wavefront per column).  The beam-frame rows that a column reads are shared with
// its neighbours in x and y, so a square patch reads about (4 + 1)^2 distinct rows
// per control point for 16 columns, where a line of four columns reads about
// 2 (4 + 1) for 4 (blocks drift apart over the control points, so rows shared
// between blocks come from beyond L2 again).  The column terms of each control
// point are computed once per block (into LDS) instead of once per voxel, and each
// lane does only the z-dependent part: the lateral coordinate j, the eight loads
// and the interpolation (the four (k, i) corners weighted first, in columns j and
// j + 1, then the step along j).  The terms are summed in control-point order with
// a compensated sum.
constexpr int GATHER_P = 4;                  // patch edge (voxel columns)
constexpr int GATHER_NW = GATHER_P * GATHER_P;  // wavefronts per block

template <typename T>
__global__ void __launch_bounds__(64 * GATHER_NW) k_gather(Geo<T> g, int nb, int first, int last, int zc, int xc,
                                                           int yc, const T* __restrict__ frame,
                                                           const T* __restrict__ mu, const T* __restrict__ Dfan,
                                                           T* __restrict__ dose, T* __restrict__ comp) {
  constexpr int NT = 64 * GATHER_NW;
  __shared__ GatherCol<T> cols[GATHER_NW][GATHER_CHUNK];
  const int nblk = zc * xc * yc;
  const int per_xcd = (nblk + 7) / 8;
  const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (w >= nblk) return;  // uniform over the block
  const int zq = w % zc, xq = (w / zc) % xc, yq = w / (zc * xc);
  const int wave = threadIdx.x >> 6;
  const int z = zq * 64 + (threadIdx.x & 63);
  const int x = xq * GATHER_P + wave % GATHER_P;
  const int y = yq * GATHER_P + wave / GATHER_P;
  const bool active = z < g.nz && x < g.nx && y < g.ny;
  const size_t vox = ((size_t)z * g.ny + y) * g.nx + x;
  const T tz = g.rel_oz + T(z) * g.sz;
  T s = T(0), c = T(0);
  if (active && !first) {
    s = dose[vox];
    c = comp[vox];
  }
  const int plane = g.Nu * g.Nv;
  const size_t cp_elems = (size_t)g.Nk * plane;
  for (int b0 = 0; b0 < nb; b0 += GATHER_CHUNK) {
    const int nbc = min(GATHER_CHUNK, nb - b0);
    __syncthreads();  // the previous chunk's column terms are no longer read
    for (int e = threadIdx.x; e < GATHER_NW * nbc; e += NT) {
      const int cw = e / nbc, bb = e - cw * nbc, b = b0 + bb;
      const T tx = g.rel_ox + T(xq * GATHER_P + cw % GATHER_P) * g.sx;
      const T ty = g.rel_oy + T(yq * GATHER_P + cw / GATHER_P) * g.sy;
      const T sn = frame[2 * b], cs = frame[2 * b + 1];
      // voxel_to_fan without the z part
      const T ev = -sn * tx + cs * ty;
      const T q = T(1) / (T(1) + ev * g.inv_sad);
      const T u = (cs * tx + sn * ty) * q;
      const T fkv = (ev - g.e0) * g.inv_dstep, fiv = u * g.inv_lat + g.cu;
      const T fk = dfloor(fkv), fi = dfloor(fiv);
      const bool in_ki = (fk >= T(-1)) & (fk < T(g.Nk)) & (fi >= T(-1)) & (fi < T(g.Nu));
      const int k0 = in_ki ? (int)fk : 0, i0 = in_ki ? (int)fi : 0;
      const T wk = fkv - fk, wi = fiv - fi;
      GatherCol<T> col;
      col.q = q;
#pragma unroll
      for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
          const int kk = k0 + dk, ii = i0 + di;
          const bool ok = in_ki & (kk >= 0) & (kk < g.Nk) & (ii >= 0) & (ii < g.Nu);
          const T wkk = dk ? wk : T(1) - wk, wii = di ? wi : T(1) - wi;
          col.w[2 * dk + di] = T(ok) * (wkk * wii);
          col.off[2 * dk + di] = min(max(kk, 0), g.Nk - 1) * plane + min(max(ii, 0), g.Nu - 1) * g.Nv;
        }
      cols[cw][bb] = col;
    }
    __syncthreads();
    if (active) {
      // the eight loads of a control point, then its term (in control-point order);
      // groups of four control points keep 32 loads in flight
      struct Term {
        T lo[4], hi[4], wj, jin0, jin1, in_j;
      };
      auto fetch = [&](int bb, Term& tm) {
        const GatherCol<T>& col = cols[wave][bb];
        const T q = uniform(col.q);
        const T fjv = tz * q * g.inv_lat + g.cv;
        const T fj = dfloor(fjv);
        const bool in_j = (fj >= T(-1)) & (fj < T(g.Nv));
        const int j0 = in_j ? (int)fj : 0;
        tm.wj = fjv - fj;
        tm.in_j = T(in_j);
        const int ja = max(j0, 0), jb = min(j0 + 1, g.Nv - 1);
        tm.jin0 = T(j0 >= 0);
        tm.jin1 = T(j0 + 1 < g.Nv);
        const T* base = Dfan + (size_t)(b0 + bb) * cp_elems;
        // 32-bit unsigned byte offsets from a scalar row address (the load's scalar base)
        const unsigned oa = (unsigned)ja * (unsigned)sizeof(T), ob = (unsigned)jb * (unsigned)sizeof(T);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const char* row = reinterpret_cast<const char*>(base + uniform(col.off[cc]));
          tm.lo[cc] = *reinterpret_cast<const T*>(row + oa);
          tm.hi[cc] = *reinterpret_cast<const T*>(row + ob);
        }
      };
      auto add = [&](int bb, const Term& tm) {
        const GatherCol<T>& col = cols[wave][bb];
        // the (k, i) corners weighted first (columns j and j + 1), then the j step
        T lo = T(0), hi = T(0);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const T w = uniform(col.w[cc]);
          lo += w * tm.lo[cc];
          hi += w * tm.hi[cc];
        }
        const T a = tm.jin0 * lo, bv = tm.jin1 * hi;
        const T acc = a + tm.wj * (bv - a);
        // outside the beam-frame grid the term is +0, which leaves s and c unchanged
        const T val = tm.in_j * (mu[b0 + bb] * acc);
        const T t = s + val;
        c += fabs(s) >= fabs(val) ? (s - t) + val : (val - t) + s;
        s = t;
      };
      int bb = 0;
      for (; bb + 4 <= nbc; bb += 4) {
        Term tm[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) fetch(bb + u, tm[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) add(bb + u, tm[u]);
      }
      for (; bb < nbc; ++bb) {
        Term tm;
        fetch(bb, tm);
        add(bb, tm);
      }
    }
  }
  if (!active) return;
  if (last) {
    dose[vox] = g.calib * (s + c);
  } else {
    dose[vox] = s;
    comp[vox] = c;
  }
}

template <typename T>
hipError_t launch_gather(const Geo<T>& g, int nb, int first, int last, const T* frame, const T* mu, const T* Dfan,
                         T* dose, T* comp, hipStream_t s) {
  const int zc = (g.nz + 63) / 64, xc = (g.nx + GATHER_P - 1) / GATHER_P, yc = (g.ny + GATHER_P - 1) / GATHER_P;
  const long nblk = (long)zc * xc * yc;
  if (nblk > 0x7ffffff0L) return hipErrorInvalidConfiguration;
  if ((long)g.Nk * g.Nu * g.Nv > 0x7fffffffL) return hipErrorInvalidConfiguration;  // 32-bit corner offsets
  const int grid = (int)((nblk + 7) / 8 * 8);
  hipLaunchKernelGGL(k_gather<T>, dim3(grid), dim3(64 * GATHER_NW), 0, s, g, nb, first, last, zc, xc, yc, frame, mu,
                     Dfan, dose, comp);
  return hipGetLastError();
}

#define PDRT_INST(T)                                                                                         \
  template hipError_t launch_frame<T>(const Geo<T>&, const T*, int, T*, hipStream_t);                        \
  template hipError_t launch_transpose_rho<T>(const Geo<T>&, const T*, T*, hipStream_t);                     \
  template hipError_t launch_raster<T>(const Geo<T>&, int, const T*, const T*, T*, hipStream_t);             \
  template hipError_t launch_aperture_box<T>(const Geo<T>&, int, const T*, int, int, int*, hipStream_t);     \
  template hipError_t launch_ca_depth<T>(const Geo<T>&, int, const T*, const T*, T*, hipStream_t);           \
  template hipError_t launch_march<T>(const Geo<T>&, int, const T*, const T*, const T*, const T*, const T*, T*, \
                                      hipStream_t, const int*);                                              \
  template hipError_t launch_march_adj<T>(const Geo<T>&, int, const T*, const T*, const T*, const T*, const T*, \
                                          T*, hipStream_t, const int*);                                      \
  template hipError_t launch_conv_direct<T>(const Geo<T>&, int, const T*, const T*, T*, hipStream_t);        \
  template hipError_t launch_gather<T>(const Geo<T>&, int, int, int, const T*, const T*, const T*, T*, T*,    \
                                       hipStream_t);

PDRT_INST(float)
PDRT_INST(double)

}  // namespace pdrt
