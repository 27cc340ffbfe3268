// dose_bwd.hip — reverse-mode kernels of the dose path and the projection layer.
//
// Given g = dL/dD the backward of one control-point batch runs
//   k_backproject_adj  Ghat_b = (trilinear back-projection)^T g   (adjoint of §2.2.7)
//   conv          H = K_k (*) Ghat_k (the taps are point symmetric, so the
//                 transposed convolution is the convolution itself; §2.2.6)
//   k_march (adjoint mode)  A = sum_k H_k (SAD/d_k)^2 DD(W_k), W recomputed (§2.2.3-2.2.4)
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
// (§2.2.7), in gather form over tiles of beam-frame columns.  A voxel contributes
// to node (k, i, j) iff its continuous indices fall in [k-1, k+1) x [i-1, i+1) x
// [j-1, j+1); (kappa, iota) depend only on the voxel's (x, y) column and jota is
// increasing in z.  One workgroup owns a tile of BT x BT columns (k, i) of one
// control point:
//   A. candidate voxel columns: the rotated box around the trapezoid of beam-frame
//      points with kappa, iota in the tile's range (plus one), each evaluated with
//      the forward's own index arithmetic and compacted in scan order;
//   B. per candidate the z sum T_c[j] = sum_z w_j(z) g(x, y, z) along its column,
//      once, shared by the up to four tile columns it touches.  The g columns of a
//      group of candidates are read with coalesced loads that are all in flight
//      together and parked in LDS before the sums read them;
//   C. each wavefront owns two rows k of the tile and adds w_k w_i T_c into them,
//      candidates in list order.
// No atomics: every sum runs in a fixed order, so the result is deterministic.
// g_t is the dose gradient in z-fastest order [ny][nx][nz].
constexpr int BP_BT = 8;      // tile edge (beam-frame columns)
constexpr int BP_CB = 32;     // candidates whose z sums are held at once
constexpr int BP_CMAX = 256;  // candidates examined per pass (one per thread)
constexpr int BP_ZREG = 16;   // g values per lane parked per group (group size x column chunks)

template <typename T, int JS>
struct BpLds {
  static constexpr int JC = 64 * JS;  // beam-frame j handled per chunk
  T tsum[BP_CB * JC];
  T acc[BP_BT * BP_BT * JC];
  T zbuf[4 * BP_ZREG * 64];           // per wavefront: a group's g columns
  T c_wk[BP_CMAX], c_wi[BP_CMAX], c_q[BP_CMAX], c_dq[BP_CMAX];
  int c_col[BP_CMAX], c_kf[BP_CMAX], c_if[BP_CMAX];
  int wcount[4];
};

// z sum of one candidate column for beam-frame j: the z whose jota lies in
// [j-1, j+1), widened by one voxel each side (the weight is zero outside).
template <typename T, typename Col>
__device__ __forceinline__ T z_sum(const Geo<T>& g, int j, T qc, T dqc, Col col) {
  const T za = ((T(j - 1) - g.cv) * g.lat * dqc - g.rel_oz) * g.inv_sz;
  const T zb = ((T(j + 1) - g.cv) * g.lat * dqc - g.rel_oz) * g.inv_sz;
  const int z0 = max(0, (int)dfloor(za) - 1), z1 = min(g.nz - 1, (int)dfloor(zb) + 1);
  T part = T(0);
  for (int z = z0; z <= z1; ++z) {
    const T tz = g.rel_oz + T(z) * g.sz;
    const T jj = tz * qc * g.inv_lat + g.cv;
    const T fj = dfloor(jj);
    const int j0 = (int)fj;
    const T wj = jj - fj;
    const T w = j0 == j ? T(1) - wj : (j0 == j - 1 ? wj : T(0));
    part += w * col(z);
  }
  return part;
}

// ZS = 64-element chunks of a g column parked in LDS (nz <= 64 ZS); ZS = 0 reads
// the columns straight from global memory (very long columns).
template <typename T, int JS, int ZS>
__global__ void __launch_bounds__(256) k_backproject_adj(Geo<T> g, int tiles_i, const T* __restrict__ frame,
                                                         const T* __restrict__ g_t, T* __restrict__ Ghat) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  BpLds<T, JS>& L = *reinterpret_cast<BpLds<T, JS>*>(smem_raw);
  constexpr int JC = BpLds<T, JS>::JC;
  constexpr int G = ZS > 0 ? BP_ZREG / ZS : 1;  // candidates per group
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b = blockIdx.y;
  const int k0 = (blockIdx.x / tiles_i) * BP_BT, i0 = (blockIdx.x % tiles_i) * BP_BT;
  const int kn = min(BP_BT, g.Nk - k0), in = min(BP_BT, g.Nu - i0);
  const T sn = frame[2 * b], cs = frame[2 * b + 1];
  // beam-frame box: e = d - SAD with kappa in [k0-1, k0+kn), lateral l = u d / SAD
  const T e_lo = g.e0 + T(k0 - 1) * g.dstep, e_hi = g.e0 + T(k0 + kn) * g.dstep;
  const T u_lo = (T(i0 - 1) - g.cu) * g.lat, u_hi = (T(i0 + in) - g.cu) * g.lat;
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
  const T eps = T(1e-3);  // rounding margin (index units); membership uses the forward's arithmetic
  const int x0 = max(0, (int)dfloor(xmin - eps) + 1), x1 = min(g.nx - 1, (int)dfloor(xmax + eps));
  const int y0 = max(0, (int)dfloor(ymin - eps) + 1), y1 = min(g.ny - 1, (int)dfloor(ymax + eps));
  const int bw = x1 - x0 + 1, nbox = (x1 >= x0 && y1 >= y0) ? bw * (y1 - y0 + 1) : 0;
  // wave w owns tile rows k0 + 2w, k0 + 2w + 1
  const int r_lo = k0 + 2 * wave, r_hi = min(k0 + kn, r_lo + 2);
  const size_t plane = (size_t)g.Nu * g.Nv;
  T* out_b = Ghat + (size_t)b * g.Nk * plane;
  T* zb_w = L.zbuf + wave * (BP_ZREG * 64);

  for (int jc0 = 0; jc0 < g.Nv; jc0 += JC) {
    for (int idx = tid; idx < BP_BT * BP_BT * JC; idx += 256) L.acc[idx] = T(0);
    for (int base = 0; base < nbox; base += BP_CMAX) {
      // A. candidates among box columns base .. base + 255, compacted in scan order
      const int idx = base + tid;
      bool is_cand = false;
      int col = 0, kf = 0, ifl = 0;
      T wk = T(0), wi = T(0), q = T(0), dq = T(0);
      if (idx < nbox) {
        const int y = y0 + idx / bw, x = x0 + idx % bw;
        const T tx = g.rel_ox + T(x) * g.sx, ty = g.rel_oy + T(y) * g.sy;
        FanIdx<T> f = voxel_to_fan(g, sn, cs, tx, ty, T(0));
        const T fk = dfloor(f.k), fi = dfloor(f.i);
        kf = (int)fk;
        ifl = (int)fi;
        is_cand = kf >= k0 - 1 && kf < k0 + kn && ifl >= i0 - 1 && ifl < i0 + in;
        wk = f.k - fk;
        wi = f.i - fi;
        const T e = -sn * tx + cs * ty;
        dq = T(1) + e * g.inv_sad;  // d / SAD
        q = T(1) / dq;              // SAD / d, as in voxel_to_fan
        col = y * g.nx + x;
      }
      const unsigned long long mask = __ballot(is_cand);
      const int before = __popcll(mask & ((1ull << lane) - 1ull));
      if (lane == 0) L.wcount[wave] = __popcll(mask);
      __syncthreads();
      int off = 0, ncand = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        off += w < wave ? L.wcount[w] : 0;
        ncand += L.wcount[w];
      }
      if (is_cand) {
        const int c = off + before;
        L.c_col[c] = col;
        L.c_kf[c] = kf;
        L.c_if[c] = ifl;
        L.c_wk[c] = wk;
        L.c_wi[c] = wi;
        L.c_q[c] = q;
        L.c_dq[c] = dq;
      }
      __syncthreads();
      for (int cb0 = 0; cb0 < ncand; cb0 += BP_CB) {
        const int cn = min(BP_CB, ncand - cb0);
        // B. z sums of this batch's candidates: wavefront w takes w, w + 4, ... in groups of G
        for (int c0 = wave; c0 < cn; c0 += 4 * G) {
          if (ZS > 0) {
            T v[G][ZS > 0 ? ZS : 1];
#pragma unroll
            for (int q = 0; q < G; ++q) {
              const int c = min(c0 + 4 * q, cn - 1);
              const T* gcol = g_t + (size_t)L.c_col[cb0 + c] * g.nz;
#pragma unroll
              for (int s = 0; s < ZS; ++s) v[q][s] = gcol[min(64 * s + lane, g.nz - 1)];
            }
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
              for (int s = 0; s < ZS; ++s) zb_w[(q * ZS + s) * 64 + lane] = v[q][s];
            __builtin_amdgcn_wave_barrier();
          }
          for (int q = 0; q < G; ++q) {
            const int c = c0 + 4 * q;
            if (c >= cn) break;
            const int cc = cb0 + c;
            const T qc = L.c_q[cc], dqc = L.c_dq[cc];
            const T* gcol = g_t + (size_t)L.c_col[cc] * g.nz;
            const T* zcol = zb_w + q * ZS * 64;
#pragma unroll
            for (int s = 0; s < JS; ++s) {
              const int j = jc0 + 64 * s + lane;
              T part = T(0);
              if (j < g.Nv) {
                if (ZS > 0)
                  part = z_sum(g, j, qc, dqc, [&](int z) { return zcol[z]; });
                else
                  part = z_sum(g, j, qc, dqc, [&](int z) { return gcol[z]; });
              }
              L.tsum[c * JC + 64 * s + lane] = part;
            }
          }
          __builtin_amdgcn_wave_barrier();  // the next group overwrites this wavefront's slice
        }
        __syncthreads();
        // C. each wavefront adds the batch into its own rows, candidates in order
        for (int c = 0; c < cn; ++c) {
          const int cc = cb0 + c;
          const int ck = L.c_kf[cc];
          if (ck + 1 < r_lo || ck >= r_hi) continue;
          const int ci = L.c_if[cc];
          const T cwk = L.c_wk[cc], cwi = L.c_wi[cc];
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int k = ck + a;
            if (k < r_lo || k >= r_hi) continue;
            const T wkk = a ? cwk : T(1) - cwk;
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
              const int i = ci + bb;
              if (i < i0 || i >= i0 + in) continue;
              const T w2 = wkk * (bb ? cwi : T(1) - cwi);
              T* dst = L.acc + ((k - k0) * BP_BT + (i - i0)) * JC;
              const T* src = L.tsum + c * JC;
#pragma unroll
              for (int s = 0; s < JS; ++s) dst[64 * s + lane] += w2 * src[64 * s + lane];
            }
          }
        }
        __syncthreads();
      }
    }
    // write the tile's columns for this j chunk
    for (int idx = tid; idx < kn * in * JC; idx += 256) {
      const int node = idx / JC, jl = idx - node * JC;
      const int kk = node / in, ii = node - kk * in;
      const int j = jc0 + jl;
      if (j < g.Nv)
        out_b[(size_t)(k0 + kk) * plane + (size_t)(i0 + ii) * g.Nv + j] = L.acc[(kk * BP_BT + ii) * JC + jl];
    }
    __syncthreads();
  }
}

// Register-tiled variant (used whenever Nv <= 256): one wavefront owns a
// BR_TK x BR_TI block of beam-frame columns (k, i) of one control point and keeps
// their Nv sums in registers (lanes along j).  Its members are the voxel columns
// with floor(kappa) in [k0-1, k0+TK) and floor(iota) in [i0-1, i0+TI), found by
// testing the voxel columns of the block's rotated bounding box 64 at a time with
// the forward's index arithmetic; each member's z sum T_c[j] (tent form below) is
// formed once and added with weight w_k w_i to the (at most four) columns of the
// block it touches.
// Members are taken in scan order and z in increasing order, so every sum has a
// fixed order; no LDS, no barriers, no atomics.
constexpr int BR_TK = 4, BR_TI = 4;

__device__ __forceinline__ float bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int bcast(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

// z sum of one member column for beam-frame j in tent form: along the column the
// continuous index jj(z) = A + B z is affine (A = rel_oz q / lat + c_v,
// B = s_z q / lat), and the trilinear weight of node j is max(0, 1 - |jj - j|);
// only the z with jj in (j - 1, j + 1), found from the inverse map, are visited.
// The z are taken four at a time, their loads issued together (addresses clamped
// to z1, weights past z1 zero, which adds exact zeros), so a lane waits once per
// four voxels rather than once per voxel; the terms keep their order.
template <typename T, typename Col>
__device__ __forceinline__ T z_sum_tent(const Geo<T>& g, int j, T A, T B, T invB, Col col) {
  const T za = (T(j - 1) - A) * invB, zb = (T(j + 1) - A) * invB;
  const int z0 = max(0, (int)dfloor(za)), z1 = min(g.nz - 1, (int)dfloor(zb));
  T part = T(0);
  for (int z = z0; z <= z1; z += 4) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = col(min(z + u, z1));
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T jj = A + T(z + u) * B;
      const T w = z + u <= z1 ? fmax(T(0), T(1) - fabs(jj - T(j))) : T(0);
      part += w * v[u];
    }
  }
  return part;
}

template <typename T, int JS>
__global__ void __launch_bounds__(256) k_backproject_reg(Geo<T> g, int nb, int tiles_k, int tiles_i, int per_xcd,
                                                         const T* __restrict__ frame, const T* __restrict__ g_t,
                                                         T* __restrict__ Ghat) {
  const int lane = threadIdx.x & 63;
  // workgroups reach the eight XCDs round robin; renumber so that each XCD walks a
  // contiguous range of blocks (neighbouring columns of the same control point)
  const int logical = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const long wid = (long)logical * 4 + (threadIdx.x >> 6);
  const long n_waves = (long)nb * tiles_k * tiles_i;
  if (wid >= n_waves) return;
  const int it = (int)(wid % tiles_i);
  const long rest = wid / tiles_i;
  const int kt = (int)(rest % tiles_k), b = (int)(rest / tiles_k);
  const int k0 = kt * BR_TK, i0 = it * BR_TI;
  const T sn = frame[2 * b], cs = frame[2 * b + 1];
  // rotated bounding box of the beam-frame points with kappa in [k0-1, k0+TK), iota in [i0-1, i0+TI)
  const T e_lo = g.e0 + T(k0 - 1) * g.dstep, e_hi = g.e0 + T(k0 + BR_TK) * g.dstep;
  const T u_lo = (T(i0 - 1) - g.cu) * g.lat, u_hi = (T(i0 + BR_TI) - g.cu) * g.lat;
  const T s_lo = T(1) + e_lo * g.inv_sad, s_hi = T(1) + e_hi * g.inv_sad;
  const T l_lo = fmin(u_lo * s_lo, u_lo * s_hi), l_hi = fmax(u_hi * s_lo, u_hi * s_hi);
  T xmin = T(1e30), xmax = T(-1e30), ymin = T(1e30), ymax = T(-1e30);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const T e = (c & 1) ? e_hi : e_lo, l = (c & 2) ? l_hi : l_lo;
    const T X = (-sn * e + cs * l - g.rel_ox) * g.inv_sx;
    const T Y = (cs * e + sn * l - g.rel_oy) * g.inv_sy;
    xmin = fmin(xmin, X);
    xmax = fmax(xmax, X);
    ymin = fmin(ymin, Y);
    ymax = fmax(ymax, Y);
  }
  const T eps = T(1e-3);  // rounding margin (index units); membership uses the forward's arithmetic
  const int x0 = max(0, (int)dfloor(xmin - eps) + 1), x1 = min(g.nx - 1, (int)dfloor(xmax + eps));
  const int y0 = max(0, (int)dfloor(ymin - eps) + 1), y1 = min(g.ny - 1, (int)dfloor(ymax + eps));
  const int bw = x1 - x0 + 1, nbox = (x1 >= x0 && y1 >= y0) ? bw * (y1 - y0 + 1) : 0;

  T acc[BR_TK][BR_TI][JS];
#pragma unroll
  for (int a = 0; a < BR_TK; ++a)
#pragma unroll
    for (int c = 0; c < BR_TI; ++c)
#pragma unroll
      for (int s = 0; s < JS; ++s) acc[a][c][s] = T(0);

  for (int base = 0; base < nbox; base += 64) {
    const int idx = base + lane;
    bool member = false;
    int col = 0, kf = 0, ifl = 0;
    T wk = T(0), wi = T(0), q = T(1), dq = T(1);
    if (idx < nbox) {
      const int y = y0 + idx / bw, x = x0 + idx % bw;
      const T tx = g.rel_ox + T(x) * g.sx, ty = g.rel_oy + T(y) * g.sy;
      FanIdx<T> f = voxel_to_fan(g, sn, cs, tx, ty, T(0));
      const T fk = dfloor(f.k), fi = dfloor(f.i);
      kf = (int)fk;
      ifl = (int)fi;
      member = kf >= k0 - 1 && kf < k0 + BR_TK && ifl >= i0 - 1 && ifl < i0 + BR_TI;
      wk = f.k - fk;
      wi = f.i - fi;
      const T e = -sn * tx + cs * ty;
      dq = T(1) + e * g.inv_sad;  // d / SAD
      q = T(1) / dq;              // SAD / d, as in voxel_to_fan
      col = y * g.nx + x;
    }
    unsigned long long mask = __ballot(member);
    while (mask) {
      const int src = __builtin_ctzll(mask);
      mask &= mask - 1ull;
      const int ck = bcast(kf, src), ci = bcast(ifl, src), cc = bcast(col, src);
      const T cwk = bcast(wk, src), cwi = bcast(wi, src), cq = bcast(q, src), cdq = bcast(dq, src);
      const T* gcol = g_t + (size_t)cc * g.nz;
      const T qi = cq * g.inv_lat;
      const T A = g.rel_oz * qi + g.cv, B = g.sz * qi, invB = cdq * g.lat * g.inv_sz;
      T part[JS];
#pragma unroll
      for (int s = 0; s < JS; ++s) {
        const int j = 64 * s + lane;
        part[s] = j < g.Nv ? z_sum_tent(g, j, A, B, invB, [&](int z) { return gcol[z]; }) : T(0);
      }
      // only the (at most) 2 x 2 block columns the member touches: the member's
      // corner (ck, ci) is wavefront-uniform, so these are scalar branches
      const int ak = ck - k0, ai = ci - i0;
#pragma unroll
      for (int a = 0; a < BR_TK; ++a) {
        if (a != ak && a != ak + 1) continue;
        const T wkk = a == ak ? T(1) - cwk : cwk;
#pragma unroll
        for (int c = 0; c < BR_TI; ++c) {
          if (c != ai && c != ai + 1) continue;
          const T w2 = wkk * (c == ai ? T(1) - cwi : cwi);
#pragma unroll
          for (int s = 0; s < JS; ++s) acc[a][c][s] += w2 * part[s];
        }
      }
    }
  }
  const size_t plane = (size_t)g.Nu * g.Nv;
  T* out_b = Ghat + (size_t)b * g.Nk * plane;
#pragma unroll
  for (int a = 0; a < BR_TK; ++a) {
    if (k0 + a >= g.Nk) break;
#pragma unroll
    for (int c = 0; c < BR_TI; ++c) {
      if (i0 + c >= g.Nu) break;
      T* o = out_b + (size_t)(k0 + a) * plane + (size_t)(i0 + c) * g.Nv;
#pragma unroll
      for (int s = 0; s < JS; ++s) {
        const int j = 64 * s + lane;
        if (j < g.Nv) o[j] = acc[a][c][s];
      }
    }
  }
}

template <typename T, int JS>
static hipError_t launch_bp_reg(const Geo<T>& g, int nb, const T* frame, const T* g_t, T* Ghat, hipStream_t s) {
  const int tiles_k = (g.Nk + BR_TK - 1) / BR_TK, tiles_i = (g.Nu + BR_TI - 1) / BR_TI;
  const long n_waves = (long)nb * tiles_k * tiles_i;
  const long blocks = (n_waves + 3) / 4;
  const long per_xcd = (blocks + 7) / 8;
  if (per_xcd * 8 > 0x7fffffffL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_backproject_reg<T, JS>), dim3((unsigned)(per_xcd * 8)), dim3(256), 0, s, g, nb, tiles_k,
                     tiles_i, (int)per_xcd, frame, g_t, Ghat);
  return hipGetLastError();
}

template <typename T, int JS, int ZS>
static hipError_t launch_bp(const Geo<T>& g, int nb, const T* frame, const T* g_t, T* Ghat, hipStream_t s) {
  const size_t lds = sizeof(BpLds<T, JS>);
  {
    hipError_t e = ensure_lds_limit((const void*)k_backproject_adj<T, JS, ZS>, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int tiles_i = (g.Nu + BP_BT - 1) / BP_BT, tiles_k = (g.Nk + BP_BT - 1) / BP_BT;
  dim3 grid(tiles_i * tiles_k, nb);
  hipLaunchKernelGGL((k_backproject_adj<T, JS, ZS>), grid, dim3(256), lds, s, g, tiles_i, frame, g_t, Ghat);
  return hipGetLastError();
}

template <typename T, int JS>
static hipError_t launch_bp_z(const Geo<T>& g, int nb, const T* frame, const T* g_t, T* Ghat, hipStream_t s) {
  if (g.nz <= 128) return launch_bp<T, JS, 2>(g, nb, frame, g_t, Ghat, s);
  if (g.nz <= 256) return launch_bp<T, JS, 4>(g, nb, frame, g_t, Ghat, s);
  if (g.nz <= 512) return launch_bp<T, JS, 8>(g, nb, frame, g_t, Ghat, s);
  return launch_bp<T, JS, 0>(g, nb, frame, g_t, Ghat, s);
}

template <typename T>
hipError_t launch_backproject_adj(const Geo<T>& g, int nb, const T* frame, const T* g_t, T* Ghat, hipStream_t s) {
  if (g.Nv <= 64) return launch_bp_reg<T, 1>(g, nb, frame, g_t, Ghat, s);
  if (g.Nv <= 128) return launch_bp_reg<T, 2>(g, nb, frame, g_t, Ghat, s);
  if (g.Nv <= 192) return launch_bp_reg<T, 3>(g, nb, frame, g_t, Ghat, s);
  if (g.Nv <= 256) return launch_bp_reg<T, 4>(g, nb, frame, g_t, Ghat, s);
  // wider planes: the LDS-tiled kernel, j in chunks of 64 or 128 (FP64: 64)
  if (sizeof(T) == 8) return launch_bp_z<T, 1>(g, nb, frame, g_t, Ghat, s);
  return launch_bp_z<T, 2>(g, nb, frame, g_t, Ghat, s);
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

__device__ __forceinline__ float dceil(float x) { return ceilf(x); }
__device__ __forceinline__ double dceil(double x) { return ceil(x); }

// First leaf pair whose upper edge lies above x (edges ascending; L if none).
template <typename T>
__device__ __forceinline__ int leaf_first(const Geo<T>& g, T x) {
  int lo = 0, hi = g.L;  // answer in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (g.leaf_edges[mid + 1] > x)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
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
  const int L = g.L;
  const T D = g.lat, iD = g.inv_lat, tau = g.tau;
  const T* jw = jaws + 4 * b;
  const T* lv = leaves + (size_t)2 * L * b;
  const T* Ab = A + (size_t)b * g.Nu * g.Nv;
  const T scale = g.calib * mu[b];
  // Every term carries fx fy or one of their jaw derivatives, which vanish on
  // pixels that do not overlap the jaw opening: only the pixels of the jaw
  // rectangle (one pixel wider each side) are visited, and for each pixel row
  // only the leaf pairs whose rows it overlaps.
  const int u0 = max(0, (int)dfloor(jw[0] * iD + g.cu - T(0.5)) - 1);
  const int u1 = min(g.Nu, (int)dceil(jw[1] * iD + g.cu + T(0.5)) + 1);
  const int v0 = max(0, (int)dfloor(jw[2] * iD + g.cv - T(0.5)) - 1);
  const int v1 = min(g.Nv, (int)dceil(jw[3] * iD + g.cv + T(0.5)) + 1);
  const bool finite = jw[0] == jw[0] && jw[1] == jw[1] && jw[2] == jw[2] && jw[3] == jw[3];
  const int iu0 = finite ? u0 : 0, iu1 = finite ? u1 : g.Nu, iv0 = finite ? v0 : 0, iv1 = finite ? v1 : g.Nv;
  const int bw = iv1 - iv0, area = iu1 > iu0 && bw > 0 ? (iu1 - iu0) * bw : 0;
  T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
  for (int rr = tid; rr < area; rr += 256) {
    const int i = iu0 + rr / bw, j = iv0 + rr % bw;
    const T u = (T(i) - g.cu) * D, v = (T(j) - g.cv) * D;
    const T fx = overlap(u, jw[0], jw[1], D, iD), fy = overlap(v, jw[2], jw[3], D, iD);
    const T dx1 = overlap_da(u, jw[0], jw[1], D, iD), dx2 = overlap_db(u, jw[0], jw[1], D, iD);
    const T dy1 = overlap_da(v, jw[2], jw[3], D, iD), dy2 = overlap_db(v, jw[2], jw[3], D, iD);
    if (fx == T(0) && fy == T(0)) continue;
    if (fx == T(0) && dx1 == T(0) && dx2 == T(0)) continue;
    if (fy == T(0) && dy1 == T(0) && dy2 == T(0)) continue;
    T S = T(0), O = T(0);
    for (int l = leaf_first(g, v - T(0.5) * D); l < L && g.leaf_edges[l] < v + T(0.5) * D; ++l) {
      const T w = overlap(v, g.leaf_edges[l], g.leaf_edges[l + 1], D, iD);
      if (w > T(0)) {
        S += w;
        O += w * overlap(u, lv[l], lv[L + l], D, iD);
      }
    }
    const T br = tau * S + (T(1) - tau) * O;
    const T a = Ab[(size_t)i * g.Nv + j];
    const T gF = scale * a;
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
  // A leaf edge's derivative lives on the pixel columns next to the edge and the
  // pixel rows the leaf pair overlaps.
  for (int t = tid; t < 2 * L; t += 256) {
    const int side = t / L, l = t - side * L;
    const T lo = lv[l], hi = lv[L + l];
    const T edge = side ? hi : lo;
    T s = T(0);
    if (edge == edge && fabs(edge) < T(1e8)) {
      const int ic = (int)dfloor(edge * iD + g.cu + T(0.5));
      const int ja = max(0, (int)dfloor(g.leaf_edges[l] * iD + g.cv - T(0.5)) - 1);
      const int jb = min(g.Nv - 1, (int)dceil(g.leaf_edges[l + 1] * iD + g.cv + T(0.5)) + 1);
      for (int j = ja; j <= jb; ++j) {
        const T v = (T(j) - g.cv) * D;
        const T w = overlap(v, g.leaf_edges[l], g.leaf_edges[l + 1], D, iD);
        if (!(w > T(0))) continue;
        const T fy = overlap(v, jw[2], jw[3], D, iD);
        if (fy == T(0)) continue;
        for (int i = max(0, ic - 1); i <= min(g.Nu - 1, ic + 1); ++i) {
          const T u = (T(i) - g.cu) * D;
          const T d = side ? overlap_db(u, lo, hi, D, iD) : overlap_da(u, lo, hi, D, iD);
          if (d == T(0)) continue;
          const T fx = overlap(u, jw[0], jw[1], D, iD);
          s += scale * Ab[(size_t)i * g.Nv + j] * fx * fy * (T(1) - tau) * w * d;
        }
      }
    } else {
      // non-finite edge: the full scan (it contributes only where its overlap derivative is defined)
      for (int j = 0; j < g.Nv; ++j) {
        const T v = (T(j) - g.cv) * D;
        const T w = overlap(v, g.leaf_edges[l], g.leaf_edges[l + 1], D, iD);
        if (!(w > T(0))) continue;
        const T fy = overlap(v, jw[2], jw[3], D, iD);
        if (fy == T(0)) continue;
        for (int i = 0; i < g.Nu; ++i) {
          const T u = (T(i) - g.cu) * D;
          const T d = side ? overlap_db(u, lo, hi, D, iD) : overlap_da(u, lo, hi, D, iD);
          if (d == T(0)) continue;
          const T fx = overlap(u, jw[0], jw[1], D, iD);
          s += scale * Ab[(size_t)i * g.Nv + j] * fx * fy * (T(1) - tau) * w * d;
        }
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
